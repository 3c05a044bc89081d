"""Throughput benchmark: full k-way partitions of a device-resident hypergraph.

One step = one complete bp_partition_device call (validation, coarsening,
initial bisection, projection + refinement at every level, every tree level
of the recursive bisection, and the final cut) on inputs already in HBM.
Prints ONE JSON line on stdout; details go to stderr.

Default workload: the netlist-shaped hypergraph (1,000,000 unit nodes,
1,200,000 hyperedges, degrees power-law 2.5 on [2,1000], 80% of pins within
+-2000 of an anchor), k = 2, eps = 0.05.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pins/sec full k-way partition (coarsen+refine) vs HBM roofline; p99 latency served"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2012_13618_amd import inputs as I
    if name == "vlsi":
        h = I.vlsi()
        desc = ("netlist-shaped: N=1,000,000 unit nodes, E=1,200,000 hyperedges, degree "
                "power-law alpha=2.5 on [2,1000], 80% of pins within +-2000 of an anchor")
    elif name == "colnet":
        h = I.column_net()
        desc = ("column-net sparse matrix: N=E=4,000,000, nnz per column power-law alpha=2.1 on "
                "[1,5000], node weight = row nnz")
    elif name == "colnet2":
        h = I.column_net(dmin=2)
        desc = ("column-net sparse matrix: N=E=4,000,000, nnz per column power-law alpha=2.1 on "
                "[2,5000], node weight = row nnz")
    elif name == "tiny":
        h = I.tiny()
        desc = "random: N=1,000 unit nodes, E=2,000 hyperedges of degree U{2..8}"
    else:
        raise SystemExit(f"unknown workload {name}")
    return h, desc


def cpu_baseline(h, k, eps, budget_s):
    """The sequential oracle, single-threaded, on the same workload."""
    import oracle
    runs, t0 = 0, time.perf_counter()
    while True:
        oracle.partition_hg(h, k=k, eps=eps)
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s or runs >= 5:
            break
    return {"value": h.num_pins * runs / el, "unit": "pins/s", "cores": 1, "kind": "oracle",
            "sample": f"{runs} full run(s) of the same workload ({h.num_pins} pins each), "
                      f"{el:.1f} s single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="vlsi")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(see the sharding plan in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2012_13618_amd as bp

    torch.cuda.set_device(0)
    h, desc = make_workload(args.workload)
    k, eps = h.meta["k"], h.meta["eps"]
    log(f"workload {args.workload}: N={h.num_nodes} E={h.num_hedges} P={h.num_pins} k={k} eps={eps}")
    dh = bp.DeviceHypergraph.from_host(h)
    part = torch.empty(h.num_nodes, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        bp.partition_device(dh, k, eps, part_out=part)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, cut, status, rep = bp.partition_device(dh, k, eps, part_out=part)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1000.0 / args.steps
    value = h.num_pins * args.steps / el
    log(f"{ms:.3f} ms/step  {value / 1e9:.3f} Gpins/s  cut={cut} status={bp.STATUS[status]}")
    log("report", json.dumps(rep.as_dict()))

    roofline = None
    if not args.no_profile:
        # one more step with per-launch hipEvent timing on the launching stream
        bp.profile_reset()
        bp.profile_enable(True)
        bp.partition_device(dh, k, eps, part_out=part)
        torch.cuda.synchronize()
        bp.profile_enable(False)
        stats = sorted(bp.profile_read(), key=lambda s: -s["total_ms"])
        tot = sum(s["total_ms"] for s in stats)
        log(f"kernel time (profiled step): {tot:.3f} ms over "
            f"{sum(s['launches'] for s in stats)} launches")
        for s in stats[:25]:
            gbs = s["bytes"] / (s["total_ms"] * 1e6) if s["total_ms"] > 0 else 0
            log(f"  {s['name']:<16} {s['launches']:6d} launches {s['total_ms']:8.3f} ms "
                f"avg {1000 * s['total_ms'] / s['launches']:8.2f} us  {gbs:8.1f} GB/s")
        dom = next((s for s in stats if s["bytes"] > 0), None)
        if dom:
            achieved = dom["bytes"] / (dom["total_ms"] * 1e6)
            roofline = {"bound": "hbm", "kernel": dom["name"], "achieved": round(achieved, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "avg_launch_us": round(1000 * dom["total_ms"] / dom["launches"], 3),
                        "launches_per_step": dom["launches"],
                        "share_of_kernel_time": round(dom["total_ms"] / tot, 4)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(h, k, eps, args.cpu_budget)
        log(f"cpu oracle: {cpu['value'] / 1e6:.3f} Mpins/s ({cpu['sample']})")

    line = {"metric": METRIC, "value": value, "unit": "pins/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic",
            "config": {"workload": desc, "nodes": h.num_nodes, "hedges": h.num_hedges,
                       "pins": h.num_pins, "k": k, "eps": eps, "parallelism": "1 GPU",
                       "cut": cut},
            "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
