"""Benchmark: connections built and indexed per second on one MI355X.

Default workload (`--workload served`): the served construction of a stream
of 10,000 uneven Connect requests (64 populations of 1e3..2e5 neurons,
request sizes log-uniform in 1e2..1e7 connections, the five rules mixed)
against a 64 GiB resident budget, then the final sort and first-index array.
One step = one whole served build of the stream; the line also reports the
per-call build of the same stream and p50/p99 per-request latency under
open-loop arrivals.

Other workloads (`--workload column8 | multiarea | collective | indegreeS |
balanced`): one step is one whole construction of one host's share of a
synthetic network: a fresh context, Create for every population, every
Connect call (generation), and Prepare (image map, remap, source-major sort,
first-index array, point-to-point and collective send lists).  Inputs are
the workload script (a few KB); everything else is built in HBM inside the
timed region.  `--workload exchange` times spike packets and delivery.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def workload(name: str, scale: float):
    from paper_2512_09502_amd import workloads as W
    if name == "column8":
        return W.column8(scale=scale)
    if name == "balanced":
        return W.balanced_small()
    if name == "multiarea":
        return W.multiarea_p2p()
    if name == "collective":
        return W.balanced_collective()
    if name.startswith("indegree"):        # indegree or indegreeS: in-degree scale S (default 2)
        return W.balanced_indegree(int(name[len("indegree"):] or 2))
    raise SystemExit(f"unknown workload {name}")


def expected_conns(script, P_local: int = 0) -> int:
    """Connections the host will hold, where the workload states it (passed to
    snnc_reserve so that the generation arrays are allocated once)."""
    info = script.get("info", {})
    if "conns_by_host" in info:
        return int(info["conns_by_host"][P_local])
    return int(info.get("conns", info.get("conns_per_host", 0)))


PHASES = (
    ("generation", ("gen_",)),
    ("keys_unique_remap", ("prep_keys", "prep_number", "prep_bits", "prep_first", "prep_fc_bits", "prep_img_list",
                           "prep_rvals", "prep_bounds", "prep_img_rows")),
    ("sort", ("sort_",)),
    ("csr", ("prep_csr",)),
    ("send_lists", ("prep_mark", "prep_tp", "prep_s_", "prep_hi", "prep_gq")),
)


def phase_times(kernels: dict, stats: dict) -> dict:
    """Kernel milliseconds of one build grouped by the path's steps (generation;
    key build, image unique/number/remap; sort; first-index array; send lists),
    and the connect and prepare phases timed by HIP events on the library stream."""
    out = {name: 0.0 for name, _ in PHASES}
    out["other"] = 0.0
    for k, (_, ms) in kernels.items():
        for name, prefixes in PHASES:
            if any(k.startswith(p) for p in prefixes):
                out[name] += ms
                break
        else:
            out["other"] += ms
    out = {k: round(v, 3) for k, v in out.items()}
    out["connect_events_ms"] = round(stats["ms_connect"], 3)
    out["prepare_events_ms"] = round(stats["ms_prepare"], 3)
    return out


def _kept(net, name) -> bool:
    """whether the prepared network holds this array (some exist at certain memory levels only)"""
    import paper_2512_09502_amd as snnc
    try:
        net.count(name)
        return True
    except snnc.SnncError:
        return False


def build_once(script, P_local: int, timing):
    import paper_2512_09502_amd as snnc
    net = snnc.Network(script["P"], P_local, script["seed"], script["dt"])
    if script.get("memory_level") is not None:
        net.set_memory_level(script["memory_level"])
    if script.get("map_policy") is not None:
        net.set_map_policy(*script["map_policy"])
    if script.get("sort_variant") is not None:
        net.tune("sort_variant", script["sort_variant"])
    for key, value in script.get("tune", {}).items():
        net.tune(key, value)
    if timing:
        net.set_timing(timing)   # 1: every launch, 2: the radix passes only
    hint = expected_conns(script, P_local)
    if hint:
        net.reserve(hint)
    for op in script["ops"]:
        if op[0] == "create":
            net.create(op[1], op[2])
        else:
            _, src, tgt, conn, syn, alpha = op
            net.connect(src, tgt, conn, syn, alpha)
    net.prepare()
    return net


# Sort + index (image map, remap, sort, first-index array, send lists):
# algorithmic bytes are one read and one write of the 14-byte connection
# record (source, target, delay, weight) per connection, 8 bytes per entry of
# the first-index array, 4 bytes per image (R), per I entry and per entry of
# the send lists (S, T, P, G, Q) plus 8 bytes per entry of their pointer arrays.
BYTES_PER_CONN = 28.0
SORT_INDEX_GROUPS = ("keys_unique_remap", "sort", "csr", "send_lists")


def index_bytes(counts: dict) -> float:
    """Algorithmic bytes of the index structures besides the connection
    records, from the element counts of the prepared arrays."""
    b = 8.0 * counts.get("row_ptr", 0)
    for k in ("r_val", "i_val", "s_val", "t_val", "p_val", "g_val", "q_val"):
        b += 4.0 * counts.get(k, 0)
    for k in ("tp_ptr", "gq_ptr"):
        b += 8.0 * counts.get(k, 0)
    return b


def measured_traffic(kernel: str, n_elem: int, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter table
    (FETCH_SIZE and WRITE_SIZE per element, calibrated), or None when no
    entry was taken on this workload or the kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        table = json.load(open(path))
        entry = next(e for e in table["entries"] if e["kernel"] == kernel and e["workload"] == workload)
        sources = entry["source"] if isinstance(entry["source"], list) else [entry["source"]]
        hashes = entry["sha1"] if isinstance(entry["sha1"], list) else [entry["sha1"]]
        current = [hashlib.sha1(open(os.path.join(ROOT, s), "rb").read()).hexdigest() for s in sources]
    except (OSError, KeyError, ValueError, StopIteration):
        return None
    if current != hashes:
        return None
    return round(n_elem * (entry["read_bytes_per_elem"] + entry["write_bytes_per_elem"]))


def sort_roofline(kt_timed: dict, breakdown: dict, n_conn: int, counts: dict, workload: str):
    """Roofline of the dominant radix pass (average launch time from the HIP
    events of the timed steps) at the sort+index figure of 28 B per
    connection, and of the whole sort+index phase (every Prepare kernel of
    the bracketed build: algorithmic bytes over their summed time)."""
    sort_like = {k: v for k, v in kt_timed.items() if k in ("sort_pass", "sort_pass_final")}
    if not sort_like or not n_conn:
        return None
    name, (launches, ms) = max(sort_like.items(), key=lambda kv: kv[1][1])
    avg_ms = ms / launches
    per_launch = BYTES_PER_CONN * n_conn
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    phase_ms = 0.0
    for k, (_, kms) in breakdown.items():
        for group, prefixes in PHASES:
            if group in SORT_INDEX_GROUPS and any(k.startswith(p) for p in prefixes):
                phase_ms += kms
                break
    phase_bytes = BYTES_PER_CONN * n_conn + index_bytes(counts)
    phase = None
    if phase_ms > 0:
        ph = phase_bytes / (phase_ms * 1e-3) / 1e9
        measured = measured_traffic("phase_sort_index", n_conn, workload)
        phase = {"kernels_ms": round(phase_ms, 3), "algorithmic_bytes": phase_bytes, "achieved": round(ph, 1),
                 "frac": round(ph / PEAK_HBM_GBS, 4),
                 "bytes_per_conn_algorithmic": round(phase_bytes / n_conn, 3),
                 "traffic": measured,
                 "bytes_per_conn_measured": round(measured / n_conn, 2) if measured else None,
                 "measured_GBs": round(measured / (phase_ms * 1e-3) / 1e9, 1) if measured else None}
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(name, n_conn, workload),
            "kernel": name, "launches_timed": launches, "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_bytes_per_launch": per_launch, "bytes_per_conn": BYTES_PER_CONN,
            "phase_sort_index": phase}


def cpu_baseline(script, budget_conns: float = 1.2e7):
    """The oracle (single-threaded C) on a bounded sample of the same
    workload: the Connect calls taken in script order while their declared
    sizes fit a connection budget, then Prepare."""
    import oracle
    ops, kept, total_calls, planned = [], 0, 0, 0
    for op in script["ops"]:
        if op[0] == "connect":
            total_calls += 1
            n = int(op[3].get("n", 0))
            if op[3]["rule"] != "fixed_total_number" or planned + n > budget_conns:
                continue
            planned += n
            kept += 1
        ops.append(op)
    sub = dict(script)
    sub["ops"] = ops
    t0 = time.perf_counter()
    net = oracle.run_script(sub, 0)
    dt = time.perf_counter() - t0
    n = int(net.array("row_ptr")[-1])
    return {"value": round(n / dt / 1e9, 6), "unit": "Gconn/s", "cores": 1, "kind": "oracle",
            "sample": f"{kept} of the {total_calls} Connect calls of the same workload, in script order while they "
                      f"fit {budget_conns:.0e} connections ({n} connections), then Prepare; {dt:.1f} s on one core"}


def exchange(args):
    """Spike exchange through the built maps of the multi-area network (one
    host's share of 32): per step, packets for the spikes of 1% of the local
    neurons (point-to-point, T/P) and delivery of received entries naming 1% of
    the images (through L into their connection rows, expanded to events)."""
    import numpy as np
    import torch
    import paper_2512_09502_amd as snnc
    script = workload("multiarea", args.scale)
    if args.memory_level is not None:
        script["memory_level"] = args.memory_level
    net = build_once(script, 0, timing=False)
    st = net.stats()
    M, n_img = st["M_local"], st["n_images"]
    r_off = net.array("r_off").astype(np.int64)
    rng = np.random.default_rng(7)
    P = script["P"]
    sizes = np.diff(r_off[: P + 1])

    def step_inputs():
        spikes = rng.choice(M, size=max(1, M // 100), replace=False).astype(np.uint32)
        k = max(1, n_img // 100)
        which = rng.choice(n_img, size=k, replace=False)
        sigma = np.searchsorted(r_off[: P + 1], which, side="right") - 1
        pos = which - r_off[sigma]
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()
        return dev(spikes), dev(sigma), dev(pos), dev(rng.integers(1, 4, size=k))

    inputs = [step_inputs() for _ in range(args.steps + args.warmup)]
    for sp, sg, ps, mu in inputs[: args.warmup]:
        net.spike_packets(0, sp)
        net.deliver(0, sg, ps, mu)
    torch.cuda.synchronize()
    net.set_timing(True)
    t_pk = t_dl = 0.0
    n_pk = n_ev = 0
    for sp, sg, ps, mu in inputs[args.warmup:]:
        t0 = time.perf_counter()
        pk = net.spike_packets(0, sp)
        t1 = time.perf_counter()
        d = net.deliver(0, sg, ps, mu)
        t2 = time.perf_counter()
        t_pk += t1 - t0
        t_dl += t2 - t1
        n_pk += int(pk["pos"].numel())
        n_ev += int(d["n_events"])
    kt = net.kernel_times()
    ev_ms = kt.get("deliver_events", (1, 0.0))
    roof = None
    if ev_ms[1] > 0:
        per_launch = 20.0 * n_ev / args.steps          # read 10 B (target, delay, weight) + write 10 B per event
        achieved = per_launch / (ev_ms[1] / ev_ms[0] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "kernel": "deliver_events",
                "avg_launch_ms": round(ev_ms[1] / ev_ms[0], 4), "algorithmic_bytes_per_launch": per_launch}
    out = {"metric": "delivered events/sec (Gevents/s) on 1 MI355X; packet entries/sec",
           "value": round(n_ev / t_dl / 1e9, 4), "unit": "Gevents/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * (t_pk + t_dl) / args.steps, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32 ids, f32 weights",
           "data": "synthetic",
           "config": {"workload": "multiarea_p2p spike exchange", "neurons": M, "images": n_img,
                      "spikes_per_step": int(inputs[0][0].numel()), "entries_per_step": int(inputs[0][1].numel()),
                      "memory_level": script.get("memory_level")},
           "packets": {"entries_per_step": n_pk // args.steps, "ms_per_step": round(1e3 * t_pk / args.steps, 3),
                       "Mentries_s": round(n_pk / t_pk / 1e6, 2)},
           "delivery": {"events_per_step": n_ev // args.steps, "ms_per_step": round(1e3 * t_dl / args.steps, 3)},
           "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in sorted(kt.items(), key=lambda kv: -kv[1][1])},
           "roofline": roof}
    net.close()
    print(json.dumps(out), flush=True)


def _cpu_info() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}


def _on_one_core(fn):
    """Run fn() with the calling thread pinned to one CPU (the first one the
    process may use); returns (result, cpu)."""
    old = os.sched_getaffinity(0)
    cpu = min(old)
    os.sched_setaffinity(0, {cpu})
    try:
        return fn(), cpu
    finally:
        os.sched_setaffinity(0, old)


def served_cpu_baseline(script, work_budget: float = 1.5e8):
    """The oracle (single-threaded C, one pinned core) on a bounded sample of
    the served stream: its first requests in submission order while their
    work (connections, plus a quarter Philox block per tested pair of the
    Bernoulli requests) fits work_budget, generated and then prepared (sort
    and first-index array).  No budget binds on this sample."""
    import oracle
    creates = [op for op in script["ops"] if op[0] == "create"]
    reqs = [op for op in script["ops"] if op[0] == "connect"]
    kept, work = [], 0.0
    for op in reqs:
        conn = op[3]
        ns, nt = sum(g[2] for g in op[1]), sum(g[2] for g in op[2])
        if conn["rule"] == "pairwise_bernoulli":
            w = conn["p"] * ns * nt + ns * nt / 4.0
        elif conn["rule"] == "fixed_indegree":
            w = nt * conn["n"]
        elif conn["rule"] == "fixed_outdegree":
            w = ns * conn["n"]
        elif conn["rule"] == "fixed_total_number":
            w = conn["n"]
        else:
            w = min(ns, nt)
        if work + w > work_budget:
            break
        work += w
        kept.append(op)
    sub = dict(script)
    sub["ops"] = creates + kept

    def run():
        t0 = time.perf_counter()
        net = oracle.run_script(sub, 0, skip_invalid=True)
        return net, time.perf_counter() - t0

    (net, dt), cpu = _on_one_core(run)
    n = int(net.array("row_ptr")[-1])
    info = _cpu_info()
    return {"value": round(n / dt / 1e9, 6), "unit": "Gconn/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {len(kept)} of the {len(reqs)} requests in submission order ({n} connections, "
                      f"{len(net.rejected)} rejected as invalid), generated and prepared (sort, first-index array) "
                      f"in {dt:.1f} s on one core (CPU {cpu} pinned)",
            **info}


def served(args):
    """Served construction of a stream of uneven Connect requests against a
    resident budget.  One step = a fresh context, Create of the 64
    populations, every request of the stream submitted in batches
    (snnc_submit_many over `batch` requests, one device wait per batch for
    the admission counts, then snnc_flush: fused generation launches), and
    the final Prepare (source-major sort and first-index array) of the
    admitted network.  The requests are marshalled into the ABI's C structs
    once, before the timed steps (they are the input).  After the timed
    steps: one per-call build of the same stream (snnc_connect per request)
    for comparison, one build with every kernel bracketed for the phase
    breakdown, and per-request latency under open-loop Poisson arrivals at
    half the measured batched capacity (one snnc_submit per arrival)."""
    import numpy as np
    import torch

    import paper_2512_09502_amd as snnc
    from paper_2512_09502_amd import workloads as W

    script = W.served_requests(n_requests=args.requests)
    budget = int(args.budget_gib * 2**30)
    creates = [op for op in script["ops"] if op[0] == "create"]
    reqs = [op for op in script["ops"] if op[0] == "connect"]
    batch = snnc.RequestBatch([op[1:] for op in reqs])

    tune = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in args.tune}

    def fresh():
        net = snnc.Network(1, 0, script["seed"], script["dt"])
        for key, val in tune.items():
            net.tune(key, val)
        net.set_resident_budget(budget)
        if args.reserve:
            net.reserve(budget // 14)
        for op in creates:
            net.create(op[1], op[2])
        return net

    def count_status(tally, status):
        if status not in (0, -1, -3, -5):
            raise snnc.SnncError(status, "request failed")
        key = {0: "admitted", -1: "invalid", -3: "over_budget", -5: "unsupported"}[status]
        tally[key] = tally.get(key, 0) + 1

    def run(mode, timing=0):
        """one build of the whole stream; timing 1 brackets every kernel
        launch, 2 the radix passes of Prepare only"""
        tally = {}
        ti = time.perf_counter()
        net = fresh()
        host_ms["init"] += 1e3 * (time.perf_counter() - ti)
        if timing == 1:
            net.set_timing(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "batched":
            for k0 in range(0, len(reqs), args.batch):
                for status, _ in net.submit_batch(batch, k0, k0 + args.batch):
                    count_status(tally, status)
                net.flush()
        else:
            for i in range(len(reqs)):
                try:
                    net.connect_packed(batch, i)
                    count_status(tally, 0)
                except snnc.SnncError as e:
                    count_status(tally, e.code)
        if timing == 2:
            net.set_timing(2)
        net.prepare()
        net.sync()
        dt = time.perf_counter() - t0
        n = net.count("src")
        st = net.stats()
        kt = net.kernel_times() if timing else {}
        tc = time.perf_counter()
        net.close()
        host_ms["close"] += 1e3 * (time.perf_counter() - tc)
        return dt, n, tally, st, kt

    # grid of the persistent batch launch from the project autotuner (untimed;
    # cached for the process, so every later context takes it at init)
    tuner = snnc.Network(1, 0, script["seed"], script["dt"])
    fused_tuning = tuner.autotune_fused(int(args.tune_conns))
    tuner.close()
    host_ms = {"init": 0.0, "close": 0.0}   # context set-up (with Create) and destroy, summed
    # warm-up (untimed): the first full-size builds also grow the allocator's pool
    for _ in range(args.warmup):
        run("batched")
    host_ms = {"init": 0.0, "close": 0.0}
    torch.cuda.synchronize()
    times, kt_total = [], {}
    n_conn, tally, stats = 0, {}, None
    t_all = time.perf_counter()
    for _ in range(args.steps):
        dt, n_conn, tally, stats, kt = run("batched", timing=2)
        times.append(dt)
        for k, (l, ms) in kt.items():
            acc = kt_total.setdefault(k, [0, 0.0])
            acc[0] += l
            acc[1] += ms
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    value = n_conn * args.steps / total / 1e9
    context_ms = {k: round(v / args.steps, 3) for k, v in host_ms.items()}

    if args.pmc_calibrate:   # outside the timed region: a copy of known size for the HBM counters
        x = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        torch.empty_like(x).copy_(x)
        torch.cuda.synchronize()
        del x
    if args.timed_only:      # profiling runs: the timed steps only
        print(json.dumps({"value": round(value, 4), "ms_per_step": round(1e3 * total / args.steps, 3),
                          "connections": n_conn, "workload": "served_requests"}), flush=True)
        return
    t_pc, n_pc, tally_pc, _, _ = run("per_call")
    assert n_pc == n_conn and tally_pc == tally, "per-call and batched builds admitted different requests"
    _, _, _, _, breakdown = run("batched", timing=1)

    # latency: open-loop arrivals at half the batched capacity
    cap = len(reqs) * args.steps / total
    lam = 0.5 * cap
    arrival = np.asarray(script["info"]["arrival"]) / lam
    net = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sojourn, service, outstanding, k, last_batch = [], [], [], 0, None
    while k < len(reqs) or outstanding:
        now = time.perf_counter() - t0
        while k < len(reqs) and arrival[k] <= now:
            ts = time.perf_counter() - t0
            try:
                cid = net.connect_packed(batch, k, submit=True)
                outstanding.append((cid, arrival[k], ts))
            except snnc.SnncError as e:
                if e.code not in (-1, -3, -5):
                    raise
            k += 1
        if outstanding and (last_batch is None or net.poll(last_batch)):
            net.flush()
            last_batch = outstanding[-1][0]
        still = []
        for cid, arr, ts in outstanding:
            if net.poll(cid):
                done = time.perf_counter() - t0
                sojourn.append(done - arr)
                service.append(done - ts)
            else:
                still.append((cid, arr, ts))
        outstanding = still
        if k < len(reqs) and not outstanding:
            time.sleep(max(0.0, min(arrival[k] - (time.perf_counter() - t0), 0.001)))
    net.prepare()
    net.close()
    soj_ms, svc_ms = np.asarray(sojourn) * 1e3, np.asarray(service) * 1e3

    roof = sort_roofline(kt_total, breakdown, n_conn, {"row_ptr": stats["M_local"] + 1}, "served_requests")
    out = {
        "metric": "connections built+indexed/sec (Gconn/s) on 1 MI355X; p50/p99 Connect latency",
        "value": round(value, 4), "unit": "Gconn/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32/u64 int + f64->f32 weights", "data": "synthetic",
        "config": {"workload": "served_requests", "requests": len(reqs), "budget_gib": args.budget_gib,
                   "populations": len(creates), "neurons": stats["M_local"],
                   "offered_connections": script["info"]["offered"], "connections": n_conn,
                   "batch": args.batch, "key_bits": stats["key_bits"], "sort_passes": stats["sort_passes"],
                   "tune": tune or None},
        "requests": tally,
        "fused_tuning": fused_tuning,
        "step_ms": {"min": round(1e3 * min(times), 3), "median": round(1e3 * sorted(times)[len(times) // 2], 3),
                    "each": [round(1e3 * t, 1) for t in times], "context_init": context_ms["init"],
                    "context_close": context_ms["close"]},
        "per_call": {"Gconn_s": round(n_pc / t_pc / 1e9, 4), "ms": round(1e3 * t_pc, 3)},
        "batched_over_per_call": round(value / (n_pc / t_pc / 1e9), 3),
        "latency": {"lambda_req_per_s": round(lam, 1), "n": int(soj_ms.size),
                    "p50_ms": round(float(np.percentile(soj_ms, 50)), 3),
                    "p99_ms": round(float(np.percentile(soj_ms, 99)), 3),
                    "service_p50_ms": round(float(np.percentile(svc_ms, 50)), 3),
                    "service_p99_ms": round(float(np.percentile(svc_ms, 99)), 3)},
        "phase_ms": phase_times(breakdown, stats),
        "kernels_ms_per_step": {k: round(v[1], 3) for k, v in sorted(breakdown.items(), key=lambda kv: -kv[1][1])},
        "roofline": roof,
        "peak_hbm_bytes": stats["bytes_peak"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = served_cpu_baseline(script)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="served",
                    help="served (default: the served request stream), column8, multiarea, collective, indegreeS, "
                         "balanced, exchange")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--tune-conns", type=float, default=1e8,
                    help="served: connections of the fused-launch autotuner's synthetic batch")
    ap.add_argument("--reserve", type=int, default=0, choices=[0, 1],
                    help="served: 0 (default) maps generation blocks as requests are admitted, 1 reserves the "
                         "whole budget up front")
    ap.add_argument("--map-policy", default=None,
                    help="numbering,sources,xi: numbering 0 canonical / 1 call order; sources 0 used / "
                         "1 threshold / 2 all passed")
    ap.add_argument("--sort-variant", type=int, default=None, help="radix-pass tile shape (snnc_tune)")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="snnc_tune setting for the build (repeatable), e.g. number_variant=10")
    ap.add_argument("--memory-level", type=int, default=None, choices=[0, 1, 2, 3],
                    help="GPU memory level: maps and image rows in host (0, 1) or device memory (2, 3)")
    ap.add_argument("--autotune", action="store_true",
                    help="run the sort autotuner in the first (untimed) warmup step")
    ap.add_argument("--timed-only", action="store_true",
                    help="served: run the timed steps only (profiling runs)")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="after the timed steps, one plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the construction of one host's share needs no second GPU "
              "(each host builds its share without communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    import numpy as np
    import paper_2512_09502_amd as snnc
    if args.workload == "served":
        return served(args)
    if args.workload == "exchange":
        return exchange(args)
    script = workload(args.workload, args.scale)
    if args.sort_variant is not None:
        script["sort_variant"] = args.sort_variant
    if args.tune:
        script["tune"] = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in args.tune}
    if args.map_policy:
        n_, s_, x_ = args.map_policy.split(",")
        script["map_policy"] = (int(n_), int(s_), float(x_))
    if args.memory_level is not None:
        script["memory_level"] = args.memory_level

    tuning = None
    for w in range(args.warmup):
        net = build_once(script, 0, timing=False)
        if w == 0 and args.autotune:
            # sort autotuner (untimed): picks the pass algorithm and tile shape for
            # this size class; later contexts in the process use its choice
            st = net.stats()
            n_w = net.count("src")
            net.close()
            tuner = snnc.Network(1, 0, 1, 0.1)
            tuning = tuner.autotune_sort(n_w, st["key_bits"])
            tuning.update({"n": n_w, "bits": st["key_bits"]})
            tuner.close()
            continue
        net.close()
    torch.cuda.synchronize()

    # timed steps (HIP events on the library stream bracket the radix passes only:
    # a bracket costs host time per launch)
    times, n_conn, kt_total, stats, counts = [], 0, {}, None, {}
    untimed = 0.0          # reporting work inside the loop that is not part of a step
    host_bytes = 0
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for step in range(args.steps):
        t0 = time.perf_counter()
        net = build_once(script, 0, timing=2)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        n_conn = net.count("src")
        stats = net.stats()
        if step == args.steps - 1:
            tq = time.perf_counter()
            host_bytes = sum(net.count(k) * np.dtype(snnc.ARRAYS[k][1]).itemsize for k in snnc.ARRAYS
                             if not k.startswith("gen_") and k != "call_off" and _kept(net, k) and net.on_host(k))
            counts = {k: net.count(k) for k in snnc.ARRAYS if not k.startswith("gen_") and _kept(net, k)}
            untimed += time.perf_counter() - tq
        for k, (l, ms) in net.kernel_times().items():
            a = kt_total.setdefault(k, [0, 0.0])
            a[0] += l
            a[1] += ms
        net.close()
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all - untimed
    # per-kernel breakdown: one more build after the timed steps, every launch bracketed
    net = build_once(script, 0, timing=1)
    breakdown = net.kernel_times()
    net.close()
    if args.pmc_calibrate:   # outside the timed region: a copy of known size for the HBM counters
        x = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        torch.empty_like(x).copy_(x)
        torch.cuda.synchronize()
        del x
    ms_per_step = 1e3 * total / args.steps
    value = n_conn * args.steps / total / 1e9

    # dominant kernel and its roofline
    per_build = breakdown or {k: (v[0] / args.steps, v[1] / args.steps) for k, v in kt_total.items()}
    dom = max(per_build.items(), key=lambda kv: kv[1][1])
    roof = sort_roofline(kt_total, per_build, n_conn, counts, script["name"])

    out = {
        "metric": "connections built+indexed/sec (Gconn/s) on 1 MI355X",
        "value": round(value, 4),
        "unit": "Gconn/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 int + f64->f32 weights",
        "data": "synthetic",
        "config": {"workload": script["name"], "connections": n_conn, "calls": stats["n_calls"],
                   "neurons": stats["M_local"], "images": stats["n_images"], "key_bits": stats["key_bits"],
                   "sort_passes": stats["sort_passes"], "scale": args.scale,
                   "map_policy": script.get("map_policy"), "memory_level": script.get("memory_level"),
                   "tune": script.get("tune")},
        "sort_tuning": tuning,
        "step_ms": {"min": round(1e3 * min(times), 3), "median": round(1e3 * sorted(times)[len(times) // 2], 3)},
        # per-phase times of the scope table's steps, from the same breakdown
        "phase_ms": phase_times(per_build, stats),
        # per-kernel breakdown of one build after the timed steps (every launch bracketed)
        "kernels_ms_per_step": {k: round(v[1], 3) for k, v in sorted(per_build.items(), key=lambda kv: -kv[1][1])},
        "dominant_kernel": dom[0],
        "roofline": roof,
        "peak_hbm_bytes": stats["bytes_peak"],
        "hbm_bytes_after_prepare": stats["bytes_live"],
        "host_bytes_after_prepare": host_bytes,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(script)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
