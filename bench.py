"""Throughput benchmark: full k-way partitions of a device-resident hypergraph.

One step = one complete bp_partition_device call (validation, coarsening,
initial bisection, projection + refinement at every level, every tree level
of the recursive bisection, and the final cut) on inputs already in HBM.
Prints ONE JSON line on stdout; details go to stderr.

Default workload: the sparse-matrix column-net hypergraph (4,000,000 rows as
nodes, 4,000,000 columns as hyperedges, nonzeros per column power-law 2.1 on
[1,5000], 16.2M pins, node weight = row nonzeros), k = 8 by recursive
bisection (three tree levels), eps = 0.03.  Other workloads: --workload
colnet2 (the same on [2,5000], 38.0M pins), vlsi (netlist-shaped, 1M nodes,
k = 2), tiny, batch, serve.
"""
import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pins/sec full k-way partition (coarsen+refine) vs HBM roofline; p99 latency served"
HBM_PEAK_GBS = 8000.0
WORKLOAD_TAG = {"vlsi": "vlsi1m_k2", "colnet": "colnet4m_k8", "colnet2": "colnet4m_pl2_k8",
                "tiny": "tiny1k_k2", "random10m": "random10m_k2", "random15m": "random15m_k2"}

# Kernel families by phase of the multilevel scheme: coarsening (Algorithms 1
# and 2 with the incidence each level needs) and uncoarsening (Algorithms 3-5:
# projection, gains, swaps, balance rounds).  The rest (validation, level-0
# copy, k-way extraction, cut) is "other".
PHASE_OF = {
    "coarsen": ["match", "match_chunks", "hedge_keys", "coarsen_init", "decode", "attach", "lead",
                "parent", "qbuild", "qbuild_block", "qbuild_huge", "dedup", "copy_pins", "classify",
                "node_ids", "hedge_ids", "incidence", "radix_hist", "radix_scatter", "level_fixup"],
    "refine": ["project", "side_weights", "gain_nodes", "gain_hedges", "gain_stats", "gain_update",
               "select", "select_pick", "seg_select", "seg_balance", "seg_initial", "balance", "flip",
               "round", "level_bound"],
}


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


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
                "[1,5000] (16.2M pins), node weight = row nnz, k=8 (3 tree levels), eps=0.03")
    elif name == "colnet2":
        h = I.column_net(dmin=2)
        desc = ("column-net sparse matrix: N=E=4,000,000, nnz per column power-law alpha=2.1 on "
                "[2,5000] (38.0M pins), node weight = row nnz, k=8 (3 tree levels), eps=0.03")
    elif name == "random10m":
        h = I.random_10m()
        desc = ("random hypergraph shaped like the paper's Random-10M: N=E=10,000,000, degree uniform "
                "in [2,21] (115M pins), unit weights, k=2, eps=0.1")
    elif name == "random15m":
        h = I.random_15m()
        desc = ("random hypergraph shaped like the paper's Random-15M: N=15,000,000, E=17,000,000, "
                "degree uniform in [2,31] (281M pins), unit weights, k=2, eps=0.1")
    elif name == "tiny":
        h = I.tiny()
        desc = "random: N=1,000 unit nodes, E=2,000 hyperedges of degree U{2..8}"
    else:
        raise SystemExit(f"unknown workload {name}")
    return h, desc


BATCH_DESC = ("batch of 256 netlist-shaped graphs: N log-uniform in [1e3, 2e5], E = 1.2 N, "
              "degree power-law alpha=2.5 on [2,1000] with 80% local pins; k = 2 for even members, "
              "4 for odd; eps = 0.05")


def cpu_baseline_batch(hs, budget_s):
    """The sequential oracle over members of the batch, in order, until the budget."""
    import oracle
    pins, runs, t0 = 0, 0, time.perf_counter()
    for h in hs:
        oracle.partition_hg(h)
        pins += h.num_pins
        runs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    cpu = host_cpu()
    return {"value": pins / el, "unit": "pins/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {runs} of the 256 members ({pins} pins), {el:.1f} s single-threaded",
            "host_nproc": cpu["nproc"], "host_cpu": cpu["model"]}


def cpu_sample(name, h):
    """A bounded sample of the workload for the oracle (10-30 s on one core):
    the workload itself, except the 38M-pin column-net, whose sample is the
    same generator at half the rows and columns (same degree law, weights, k
    and eps)."""
    from paper_2012_13618_amd import inputs as I
    if name in ("random10m", "random15m"):
        big = name == "random15m"
        n, e = (1_000_000, 1_133_333) if big else (1_000_000, 1_000_000)
        s = I.uniform_hypergraph(n, e, 2, 31 if big else 21, 6 + big, name="sample")
        s.meta.update(k=2, eps=0.1)
        return s, (f"one full k=2 partition of the same generator at a fifteenth / tenth of the size "
                   f"(N={n}, E={e}, {s.num_pins} pins)")
    if name == "colnet2":
        s = I.column_net(n=2_000_000, dmin=2)
        return s, (f"one full k={s.meta['k']} partition of the same column-net generator at half size "
                   f"(N=E=2,000,000, {s.num_pins} pins)")
    return h, f"full k={h.meta['k']} partition(s) of the workload itself ({h.num_pins} pins each)"


def cpu_baseline(name, h, k, eps, budget_s):
    """The sequential oracle as it stands, single-threaded, on a bounded sample."""
    import oracle
    s, what = cpu_sample(name, h)
    runs, t0 = 0, time.perf_counter()
    while True:
        oracle.partition_hg(s, k=k, eps=eps)
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s or runs >= 5:
            break
    cpu = host_cpu()
    return {"value": s.num_pins * runs / el, "unit": "pins/s", "cores": 1, "kind": "oracle",
            "sample": f"{runs} x {what}, {el:.1f} s on one thread",
            "host_nproc": cpu["nproc"], "host_cpu": cpu["model"]}


# Kernel families and the device functions that implement them (for matching
# hardware-counter summaries, which name device functions).
FAMILY_KERNEL = {"gain_nodes": "k_gain_nodes", "gain_hedges": "k_gain_hedges", "select": "k_select_pass",
                 "seg_select": "k_seg_select", "gain_update": "k_gain_update", "seg_balance": "k_seg_fused",
                 "seg_initial": "k_seg_fused"}


def sources_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, family):
    """HBM bytes per launch of a kernel family from the committed counter
    summary of this workload, or None when there is none or the kernel
    sources changed since the counters were taken."""
    kern = FAMILY_KERNEL.get(family)
    if not kern:
        return None
    path = os.path.join(ROOT, "profiles", f"{workload}_{family}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel") != kern or sources_sha256(d["kernel_sources"]) != d["sources_sha256"]:
        return None
    return d["hbm_bytes_per_launch"]


def profiled_step(step, workload=None):
    """One more step with per-launch hipEvent timing on the launching stream.
    The dominant kernel family is the one with the most device time once the
    per-launch cost of the event timing itself (timed on empty launches) is
    set aside; its roofline entry uses the raw event-timed average."""
    import torch
    import paper_2012_13618_amd as bp
    bp.profile_reset()
    bp.profile_enable(True)
    step()
    torch.cuda.synchronize()
    bp.profile_floor(200)
    torch.cuda.synchronize()
    bp.profile_enable(False)
    allst = bp.profile_read()
    floor = next((s for s in allst if s["name"] == "event_floor"), None)
    floor_ms = floor["total_ms"] / floor["launches"] if floor else 0.0
    stats = [s for s in allst if s["name"] != "event_floor"]
    corr = lambda s: s["total_ms"] - s["launches"] * floor_ms
    stats.sort(key=lambda s: -corr(s))
    tot = sum(s["total_ms"] for s in stats)
    log(f"kernel time (profiled step): {tot:.3f} ms over "
        f"{sum(s['launches'] for s in stats)} launches; event floor {1000 * floor_ms:.2f} us/launch")
    for s in stats[:25]:
        gbs = s["bytes"] / (s["total_ms"] * 1e6) if s["total_ms"] > 0 else 0
        log(f"  {s['name']:<16} {s['launches']:6d} launches {s['total_ms']:8.3f} ms "
            f"(net {corr(s):8.3f}) avg {1000 * s['total_ms'] / s['launches']:8.2f} us  {gbs:8.1f} GB/s "
            f"{s['bytes'] / s['launches']:12.0f} B/launch")
    phases = {}
    for ph, fams in PHASE_OF.items():
        sel = [s for s in stats if s["name"] in fams]
        b = sum(s["bytes"] for s in sel)
        t = sum(s["total_ms"] for s in sel)
        n = sum(s["launches"] for s in sel)
        gbs = b / (t * 1e6) if t > 0 else 0.0
        phases[ph] = {"algorithmic_bytes": round(b), "kernel_ms": round(t, 3), "launches": n,
                      "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"phase {ph}: {b / 1e9:.3f} GB algorithmic over {t:.3f} ms of kernel time in {n} launches "
            f"= {gbs:.1f} GB/s ({100 * gbs / HBM_PEAK_GBS:.2f}% of peak)")
    dom = next((s for s in stats if s["bytes"] > 0), None)
    if not dom:
        return None
    avg_s = dom["total_ms"] / dom["launches"] / 1e3
    per_launch = dom["bytes"] / dom["launches"]
    achieved = per_launch / avg_s / 1e9
    tr = measured_traffic(workload, dom["name"]) if workload else None
    return {"bound": "hbm", "kernel": dom["name"], "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            # HBM bytes per launch from the hardware counters, and as a rate
            "traffic": None if tr is None else round(tr),
            "traffic_gbs": None if tr is None else round(tr / avg_s / 1e9, 1),
            "algorithmic_bytes_per_launch": round(per_launch),
            "avg_launch_us": round(1e6 * avg_s, 3), "event_floor_us": round(1000 * floor_ms, 3),
            "launches_per_step": dom["launches"],
            "share_of_kernel_time": round(dom["total_ms"] / tot, 4),
            # per phase: algorithmic bytes counted per launch over event-timed kernel time
            "phases": phases}


def bench_batch(args):
    """One step = one bp_partition_batch_device call over the 256-graph batch."""
    import torch
    import paper_2012_13618_amd as bp
    from paper_2012_13618_amd import inputs as I
    hs = [I.batch_member(i) for i in range(256)]
    ks = [h.meta["k"] for h in hs]
    es = [h.meta["eps"] for h in hs]
    pins = sum(h.num_pins for h in hs)
    log(f"workload batch: 256 graphs, N={sum(h.num_nodes for h in hs)} P={pins}")
    dev = [bp.DeviceHypergraph.from_host(h) for h in hs]
    outs = [torch.empty(max(h.num_nodes, 1), dtype=torch.int32, device="cuda") for h in hs]
    torch.cuda.synchronize()
    sched = None
    if args.autotune:
        best, best_ms = bp.autotune_batch_device(dev, ks, es)
        bp.schedule_set(best)
        sched = best.as_dict()
        log(f"autotuned schedule {sched} ({best_ms:.3f} ms in the tuner)")
    run = lambda: bp.partition_batch_device(dev, ks, es, parts_out=outs)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, cuts, status, reps = run()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1000.0 / args.steps
    value = pins * args.steps / el
    log(f"{ms:.3f} ms/step  {value / 1e9:.3f} Gpins/s  total cut={sum(cuts)} "
        f"status={bp.STATUS[status]} launches={reps[0].kernel_launches} syncs={reps[0].host_syncs}")
    seq_ms = None
    if not args.no_compare:
        # the same graphs one call at a time, for comparison
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(256):
            bp.partition_device(dev[i], ks[i], es[i], part_out=outs[i])
        torch.cuda.synchronize()
        seq_ms = (time.perf_counter() - t1) * 1000.0
        log(f"one call per graph: {seq_ms:.3f} ms for the 256 graphs ({ms / seq_ms:.3f} of it batched)")
    roofline = None if args.no_profile else profiled_step(run, "batch256")
    cpu = None if args.no_cpu_baseline else cpu_baseline_batch(hs, args.cpu_budget)
    if cpu:
        log(f"cpu oracle: {cpu['value'] / 1e6:.3f} Mpins/s ({cpu['sample']})")
    line = {"metric": METRIC, "value": value, "unit": "pins/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic",
            "config": {"workload": BATCH_DESC, "graphs": 256, "pins": pins, "parallelism": "1 GPU",
                       "one_call_per_graph_ms": None if seq_ms is None else round(seq_ms, 3), "total_cut": sum(cuts),
                       "schedule": sched if sched else bp.schedule_get().as_dict()},
            "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


SERVE_DESC = ("served stream: open-loop Poisson arrivals; request pins log-uniform in [1e4, 2e6], "
              "netlist-shaped, N = pins / (1.2 x 4.54), E = 1.2 N, k uniform in {2, 4, 16}, eps = 0.05")


def _pct(x, q):
    import numpy as np
    return round(float(np.percentile(np.asarray(x), q)), 3)


def serve_fifo_plain(reqs, arrivals):
    """The same stream solved one request at a time, in arrival order, on the
    plain path (host arrays in, host arrays out, as a request is): latency =
    completion - scheduled arrival."""
    import paper_2012_13618_amd as bp
    lat = []
    t0 = time.perf_counter()
    for h, a in zip(reqs, arrivals):
        d = t0 + a - time.perf_counter()
        if d > 0:
            time.sleep(d)
        bp.partition(h.num_nodes, h.offsets, h.pins, h.meta["k"], h.meta["eps"])
        lat.append(1000.0 * (time.perf_counter() - t0 - a))
    return lat, time.perf_counter() - t0


def serve_served(reqs, arrivals, args):
    """The stream into the server: a feeder submits at the arrival times,
    the requests are collected as they complete; latency = completion -
    scheduled arrival."""
    import threading
    import paper_2012_13618_amd as bp
    R = len(reqs)
    with bp.Server(hbm_budget_bytes=args.budget_gib << 30, max_slots=args.slots, workers=args.workers,
                   max_run_pins=args.run_pins) as srv:
        tickets, subs = [None] * R, [0.0] * R
        t0 = time.perf_counter()

        def feeder():
            for i, h in enumerate(reqs):
                d = t0 + arrivals[i] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                subs[i] = time.perf_counter()
                tickets[i] = srv.submit(h)

        th = threading.Thread(target=feeder)
        th.start()
        stats = []
        for i in range(R):
            while tickets[i] is None:
                time.sleep(0.0002)
            stats.append(srv.wait(tickets[i])[3])
        th.join()
        el = time.perf_counter() - t0
    lat = [1000.0 * (subs[i] - t0 - arrivals[i]) + stats[i].latency_ms for i in range(R)]
    return lat, el, [s.batch_size for s in stats]


def bench_serve(args):
    """Open-loop Poisson streams at fractions of the plain path's capacity
    (1 / mean plain solve time), into the server and, for comparison, solved
    FIFO one at a time on the plain path; pins/s over the makespan and
    latency percentiles for both."""
    import numpy as np
    import paper_2012_13618_amd as bp
    from paper_2012_13618_amd import inputs as I
    R = args.requests
    reqs = [I.serve_request(r) for r in range(R)]
    pins = sum(h.num_pins for h in reqs)
    log(f"workload serve: {R} requests, {pins} pins")
    for h in reqs[:args.warmup]:
        bp.partition(h.num_nodes, h.offsets, h.pins, h.meta["k"], h.meta["eps"])
    t = []
    for h in reqs:
        t0 = time.perf_counter()
        bp.partition(h.num_nodes, h.offsets, h.pins, h.meta["k"], h.meta["eps"])
        t.append(time.perf_counter() - t0)
    capacity = 1.0 / float(np.mean(t))
    log(f"plain solve: mean {1000 * np.mean(t):.2f} ms -> capacity {capacity:.1f} requests/s, "
        f"{pins / sum(t) / 1e6:.1f} Mpins/s back to back")
    loads = []
    for frac in [float(x) for x in args.loads.split(",")]:
        rate = frac * capacity
        arrivals = I.poisson_arrivals(R, rate)
        lat_s, el_s, bsz = serve_served(reqs, arrivals, args)
        lat_f, el_f = serve_fifo_plain(reqs, arrivals)
        row = {"load": frac, "rate_per_s": round(rate, 3),
               "served": {"pins_per_s": pins / el_s, "p50_ms": _pct(lat_s, 50), "p99_ms": _pct(lat_s, 99),
                          "mean_batch": round(float(np.mean(bsz)), 3)},
               "fifo_plain": {"pins_per_s": pins / el_f, "p50_ms": _pct(lat_f, 50), "p99_ms": _pct(lat_f, 99)}}
        log(f"load {frac}: served {pins / el_s / 1e6:.1f} Mpins/s p50 {row['served']['p50_ms']} ms "
            f"p99 {row['served']['p99_ms']} ms | FIFO plain {pins / el_f / 1e6:.1f} Mpins/s "
            f"p50 {row['fifo_plain']['p50_ms']} ms p99 {row['fifo_plain']['p99_ms']} ms")
        loads.append(row)
    top = loads[-1]
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n_or, p_or, t0 = 0, 0, time.perf_counter()
        for h in reqs:
            oracle.partition_hg(h)
            n_or += 1
            p_or += h.num_pins
            if time.perf_counter() - t0 >= args.cpu_budget:
                break
        el = time.perf_counter() - t0
        hc = host_cpu()
        cpu = {"value": p_or / el, "unit": "pins/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {n_or} requests of the stream solved one after another, {el:.1f} s",
               "host_nproc": hc["nproc"], "host_cpu": hc["model"]}
    line = {"metric": METRIC, "value": top["served"]["pins_per_s"], "unit": "pins/s", "n_gpus": 1,
            "steps": R, "warmup": args.warmup, "ms_per_step": 1000.0 / top["rate_per_s"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic",
            "config": {"workload": SERVE_DESC, "requests": R, "pins": pins, "parallelism": "1 GPU",
                       "plain_capacity_per_s": round(capacity, 3), "budget_gib": args.budget_gib,
                       "max_slots": args.slots, "workers": args.workers, "max_run_pins": args.run_pins},
            "latency_ms": {"p50": top["served"]["p50_ms"], "p99": top["served"]["p99_ms"]},
            "loads": loads, "roofline": None, "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


def bench_ksweep(args):
    """Time against k (Section 4.4 and its figure of time over k): the same
    graph partitioned into k = 2, 4, 8, 16, 32 parts.  Every tree level of the
    recursive bisection is one pass over all of its subgraphs, so the time
    should grow with the tree depth ceil(log2 k) rather than with k."""
    import numpy as np
    import torch
    import paper_2012_13618_amd as bp
    h, desc = make_workload(args.workload_of)
    dh = bp.DeviceHypergraph.from_host(h)
    part = torch.empty(h.num_nodes, dtype=torch.int32, device="cuda")
    eps = h.meta["eps"]
    rows = []
    for k in (2, 4, 8, 16, 32):
        for _ in range(args.warmup):
            bp.partition_device(dh, k, eps, part_out=part)
        ts = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, cut, st, rep = bp.partition_device(dh, k, eps, part_out=part)
            torch.cuda.synchronize()
            ts.append(1000.0 * (time.perf_counter() - t0))
        ms = float(np.median(ts))
        rows.append({"k": k, "tree_levels": rep.tree_levels, "ms": round(ms, 3), "cut": cut,
                     "pins_per_s": h.num_pins / ms * 1000.0, "balanced": rep.balanced,
                     "launches": rep.kernel_launches})
        log(f"k={k:3d} depth {rep.tree_levels}: {ms:8.3f} ms  cut {cut}  balanced {rep.balanced}")
    d = np.array([r["tree_levels"] for r in rows], float)
    t = np.array([r["ms"] for r in rows])
    A = np.vstack([np.ones_like(d), d]).T
    coef, *_ = np.linalg.lstsq(A, t, rcond=None)
    pred = A @ coef
    r2 = 1.0 - float(np.sum((t - pred) ** 2) / np.sum((t - t.mean()) ** 2))
    log(f"time ~ {coef[0]:.3f} + {coef[1]:.3f} * ceil(log2 k) ms, R^2 {r2:.4f}")
    own = next(r for r in rows if r["k"] == h.meta["k"]) if h.meta["k"] in (2, 4, 8, 16, 32) else rows[0]
    line = {"metric": METRIC, "value": own["pins_per_s"], "unit": "pins/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": own["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": desc, "study": "time against k", "pins": h.num_pins},
            "sweep": rows, "fit_ms": {"intercept": round(float(coef[0]), 3), "per_tree_level": round(float(coef[1]), 3),
                                      "r2": round(r2, 4)},
            "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def bench_design(args):
    """The design space of Section 4.3 (its table of best settings and the
    cut-time trade-off figure): matching policy x coarsening level limit x
    refinement iterations on one graph; every setting's time and cut, and the
    Pareto frontier (no other setting both faster and of smaller cut)."""
    import numpy as np
    import torch
    import paper_2012_13618_amd as bp
    h, desc = make_workload(args.workload_of)
    dh = bp.DeviceHypergraph.from_host(h)
    part = torch.empty(h.num_nodes, dtype=torch.int32, device="cuda")
    k, eps = h.meta["k"], h.meta["eps"]
    names = {bp.LDH: "LDH", bp.HDH: "HDH", bp.RAND: "RAND", bp.LWD: "LWD", bp.HWD: "HWD"}
    rows = []
    for pol in (bp.LDH, bp.HDH, bp.RAND):
        for lv in (5, 10, 15, 25):
            for it in (0, 1, 2, 4):
                prm = bp.params(policy=pol, max_levels=lv, refine_iters=it)
                bp.partition_device(dh, k, eps, prm=prm, part_out=part)
                ts = []
                for _ in range(args.steps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, cut, st, rep = bp.partition_device(dh, k, eps, prm=prm, part_out=part)
                    torch.cuda.synchronize()
                    ts.append(1000.0 * (time.perf_counter() - t0))
                rows.append({"policy": names[pol], "max_levels": lv, "refine_iters": it,
                             "ms": round(float(np.median(ts)), 3), "cut": cut, "balanced": rep.balanced})
                log(f"{names[pol]:4s} levels {lv:2d} iters {it}: {rows[-1]['ms']:8.3f} ms cut {cut}")
    front = []
    for r in sorted(rows, key=lambda r: (r["ms"], r["cut"])):
        if r["balanced"] and (not front or r["cut"] < front[-1]["cut"]):
            front.append(r)
    log("Pareto frontier: " + "; ".join(f"{r['policy']}/{r['max_levels']}/{r['refine_iters']} "
                                        f"{r['ms']} ms cut {r['cut']}" for r in front))
    default = next(r for r in rows if r["policy"] == "LDH" and r["max_levels"] == 25 and r["refine_iters"] == 2)
    line = {"metric": METRIC, "value": h.num_pins / default["ms"] * 1000.0, "unit": "pins/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": default["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": desc, "study": "policy x level limit x refinement iterations",
                       "pins": h.num_pins, "k": k, "eps": eps},
            "sweep": rows, "pareto": front, "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


# ---- rocprofv3 summaries (the files under profiles/) ------------------------

KERNEL_SOURCES = ["paper_2012_13618_amd/csrc/" + f for f in (
    "balance.hpp", "batch.hpp", "coarsen.hpp", "common.hpp", "engine.hip", "engine.hpp", "kway.hpp",
    "level.hpp", "refine.hpp", "scan.hpp", "sched.hpp", "server.hpp", "transpose.hpp", "uncoarsen.hpp")]


def _read_csv(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _short(name):
    """A kernel's name without its parameter list and namespace."""
    n = name[5:] if name.startswith("void ") else name
    depth, out = 0, ""
    for ch in n:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out += ch
    return out.replace("bp::", "")


def summarize_stats(args):
    """Markdown summary of a rocprofv3 --stats kernel table."""
    rows = _read_csv(args.summarize_stats)
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    per = args.summary_steps
    lines = [f"# Kernel time, {args.summary_title}", "",
             "Command (from the repository root; rocprofv3 run after `cd /tmp && export TMPDIR=/tmp`, "
             "paths given absolute):", "", "    " + args.summary_command, "",
             f"rocprofv3 --stats summary; the program ran {per} partition steps (warmup, timed and one "
             f"hipEvent-profiled step), so per-step figures are totals / {per}.", "",
             f"Total kernel time: {tot / 1e6:.3f} ms  ({tot / 1e6 / per:.3f} ms per step)", "",
             "| kernel | calls | calls/step | total ms | ms/step | avg us | min us | max us | % |",
             "|---|---|---|---|---|---|---|---|---|"]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows[:args.summary_top]:
        t = float(r["TotalDurationNs"])
        c = int(r["Calls"])
        lines.append(f"| {_short(r['Name'])} | {c} | {c / per:.1f} | {t / 1e6:.3f} | {t / 1e6 / per:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {100 * t / tot:.2f} |")
    with open(args.summary_out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    log("wrote", args.summary_out)


def summarize_traffic(args):
    """HBM bytes per dispatch of one kernel family from two rocprofv3 --pmc
    runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what
    the counter reads for the 1 GiB device copy that --calibrate-copy runs."""
    fetch_csv, write_csv = args.summarize_traffic
    out = {"kernel": args.summary_kernel}

    def one(path, counter):
        rows = [r for r in _read_csv(path) if r["Counter_Name"] == counter]
        ks = [float(r["Counter_Value"]) for r in rows if args.summary_kernel in r["Kernel_Name"]]
        cp = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        return ks, cp

    fk, fc = one(fetch_csv, "FETCH_SIZE")
    wk, wc = one(write_csv, "WRITE_SIZE")
    gib = 1 << 30
    ff = gib / (max(fc) * 1024.0)
    wf = gib / (max(wc) * 1024.0)
    fpd, wpd = sum(fk) / len(fk), sum(wk) / len(wk)
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    out.update({"dispatches": len(fk), "fetch_kib_per_dispatch_raw": fpd, "write_kib_per_dispatch_raw": wpd,
                "copy_calibration": {"bytes": gib, "fetch_kib_raw": max(fc), "write_kib_raw": max(wc),
                                     "fetch_factor": ff, "write_factor": wf},
                "hbm_bytes_per_launch": fpd * 1024.0 * ff + wpd * 1024.0 * wf,
                "fetch_bytes_per_launch": fpd * 1024.0 * ff, "write_bytes_per_launch": wpd * 1024.0 * wf,
                "kernel_sources": KERNEL_SOURCES, "sources_sha256": h.hexdigest(),
                "commands": args.summary_command.split(" ;; ")})
    if args.summary_log:
        # the family's algorithmic bytes per launch, from the per-family table
        # that the profiled step of a plain run of the same workload logged
        alg = None
        pat = re.compile(r"^\s*(\S+)\s+(\d+) launches\s+([\d.]+) ms .*?([\d.]+) GB/s(?:\s+(\d+) B/launch)?")
        with open(args.summary_log) as fh:
            for line in fh:
                m = pat.match(line)
                if m and m.group(1) == args.summary_family:
                    n, ms, gbs = int(m.group(2)), float(m.group(3)), float(m.group(4))
                    alg = float(m.group(5)) if m.group(5) else gbs * ms * 1e6 / n
        if alg:
            out["family"] = args.summary_family
            out["algorithmic_bytes_per_launch"] = round(alg)
            out["traffic_over_algorithmic"] = round(out["hbm_bytes_per_launch"] / alg, 3)
    with open(args.summary_out, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    log("wrote", args.summary_out, f"{out['hbm_bytes_per_launch']:.0f} B per launch over {len(fk)} dispatches")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="colnet",
                    help="colnet (default), colnet2, vlsi, tiny, random10m, random15m, batch, serve, "
                         "ksweep, design")
    ap.add_argument("--of", dest="workload_of", default="vlsi",
                    help="ksweep / design: the graph they run on (vlsi, colnet, ...)")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (a known-size kernel "
                         "for scaling hardware byte counters)")
    ap.add_argument("--autotune", action="store_true",
                    help="batch: pick the launch schedule with the autotuner first")
    ap.add_argument("--no-compare", action="store_true",
                    help="batch: skip timing the graphs one call at a time")
    ap.add_argument("--requests", type=int, default=200, help="serve: requests in the stream")
    ap.add_argument("--loads", default="0.5,0.7,0.9,1.5",
                    help="serve: arrival rates as fractions of the plain path's capacity")
    ap.add_argument("--budget-gib", type=int, default=128, help="serve: admission budget")
    ap.add_argument("--slots", type=int, default=256, help="serve: most requests per run")
    ap.add_argument("--workers", type=int, default=4, help="serve: runs in flight at once")
    ap.add_argument("--run-pins", type=int, default=4 << 20, help="serve: input pins per run")
    ap.add_argument("--summarize-stats", metavar="CSV", help="write a profiles/ summary of a rocprofv3 "
                    "kernel_stats.csv instead of benchmarking")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write a profiles/ HBM traffic summary from two rocprofv3 --pmc runs")
    ap.add_argument("--summary-kernel", default="k_seg_select")
    ap.add_argument("--summary-title", default="")
    ap.add_argument("--summary-command", default="")
    ap.add_argument("--summary-steps", type=int, default=1)
    ap.add_argument("--summary-top", type=int, default=30)
    ap.add_argument("--summary-out", default="")
    ap.add_argument("--summary-log", default="", help="bench log whose profiled-step table gives the "
                    "family's algorithmic bytes per launch")
    ap.add_argument("--summary-family", default="seg_select")
    args = ap.parse_args()
    if args.summarize_stats:
        return summarize_stats(args)
    if args.summarize_traffic:
        return summarize_traffic(args)
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(see the sharding plan in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2012_13618_amd as bp

    torch.cuda.set_device(0)
    if args.calibrate_copy > 0:
        n = args.calibrate_copy << 18  # int32 elements
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {4 * n} bytes read, {4 * n} bytes written")
        del src, dst
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "ksweep":
        return bench_ksweep(args)
    if args.workload == "design":
        return bench_design(args)
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
        roofline = profiled_step(lambda: bp.partition_device(dh, k, eps, part_out=part),
                                 WORKLOAD_TAG.get(args.workload))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, h, k, eps, args.cpu_budget)
        log(f"cpu oracle: {cpu['value'] / 1e6:.3f} Mpins/s ({cpu['sample']})")

    line = {"metric": METRIC, "value": value, "unit": "pins/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic",
            "config": {"workload": desc, "name": args.workload, "nodes": h.num_nodes, "hedges": h.num_hedges,
                       "pins": h.num_pins, "k": k, "eps": eps, "parallelism": "1 GPU",
                       "cut": cut},
            "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
