"""Writes fullsize_oracle.json: the sequential oracle's result on the full-size
column-net workloads, for GPU parity tests whose oracle run would take minutes.

Calls only the oracle and the seeded input generators.  For each workload it
stores the cut, every part's node count and weight, the SHA-256 of the part
vector (int32 little-endian) and the part ids of every 10007th node.
Run from the repository root:  python tests/golden/make_fullsize_oracle.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2012_13618_amd import inputs as I  # noqa: E402

STRIDE = 10007

WORKLOADS = {
    "colnet4m_d1_k8": lambda: I.column_net(),
    "colnet4m_d2_k8": lambda: I.column_net(dmin=2),
}


def summarise(h, part, cut):
    k = h.meta["k"]
    part = np.ascontiguousarray(part, dtype="<i4")
    return {
        "nodes": h.num_nodes, "hedges": h.num_hedges, "pins": h.num_pins,
        "k": k, "eps": h.meta["eps"], "cut": int(cut),
        "part_sizes": np.bincount(part, minlength=k).tolist(),
        "part_weights": np.bincount(part, weights=h.node_w, minlength=k).astype(np.int64).tolist(),
        "sha256": hashlib.sha256(part.tobytes()).hexdigest(),
        "sample_stride": STRIDE, "sample": part[::STRIDE].tolist(),
    }


def main():
    out = {}
    for name, make in WORKLOADS.items():
        h = make()
        t0 = time.time()
        part, cut = oracle.partition_hg(h)
        print(f"{name}: {h.num_pins} pins, cut {cut}, oracle {time.time() - t0:.1f} s", flush=True)
        out[name] = summarise(h, part, cut)
    path = os.path.join(ROOT, "tests", "golden", "fullsize_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, separators=(",", ":"))
        fh.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
