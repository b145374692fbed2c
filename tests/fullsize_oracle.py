"""Full-size parity harness -- TEST INFRASTRUCTURE.

It runs the oracle (the plain single-threaded C in ``oracle/``) in worker
processes, each on its own share of the work, and reassembles exactly what
one oracle run over the whole network gives, so that the library's arrays at
the benchmark sizes can be compared element by element.  It imports only the
oracle and numpy; no value it computes comes from the library.

Phase A (one work item = a range of primary ordinals of one call, see
``OracleNet.call_range``): the oracle generates the range (source ordinal,
target, element, weight, delay, in canonical order (call, e)); each source
becomes its *prefix* -- its local id for a source on this host, else
M_local + (alpha + 1) G + global id -- which orders sources exactly as the
prepared network does (local neurons first, then images in (alpha + 1,
sigma, s) order).  Records are split by fixed-width prefix buckets (a stable
split, so canonical order holds inside a bucket) and stored on disk.

Round U (one task = a run of consecutive buckets): the sorted unique remote
prefixes of the task's range.  Together they are the image map: image index
= M_local + rank of the prefix among all used remote prefixes (canonical
numbering), R / L / img_base per (alpha + 1, sigma).

Phase B (same tasks): the task's records from every item, concatenated in
item order (= canonical order), mapped to source' and sorted stably by
(source', target) -- the sorted connections of that source' range -- and
compared with the library's arrays of the same range, with the row counts.

Send lists: S_tau = sorted unique local sources of tau's share of the
point-to-point calls (regenerated on tau), T/P its transpose; the collective
H = union of the source segments per (group, host), I = image index or -1,
G/Q = (group, position in H_{group,P_local}) per local source.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor

import multiprocessing as mp
import numpy as np

NB = 4096                   # prefix buckets
ITEM_RECORDS = 20_000_000   # records per work item (about)
TASK_RECORDS = 30_000_000   # records per compare task (about)


# ---------------------------------------------------------------- structure of a script
class Layout:
    """Neurons per host, global id bases, map indices and the segment tables
    of every declared call, for host P_local."""

    def __init__(self, script: dict, P_local: int, calls: list):
        P = script["P"]
        M = [0] * P
        for op in script["ops"]:
            if op[0] == "create":
                M[op[1]] += op[2]
        self.P, self.P_local, self.M = P, P_local, M
        self.M_local = M[P_local]
        self.host_base = np.concatenate([[0], np.cumsum(M)]).astype(np.int64)
        self.G = int(self.host_base[-1])
        self.calls = calls
        self.n_a = max([-1] + [int(op[5]) for op in calls]) + 2
        self.pmax = self.M_local + self.n_a * self.G
        self.segs = []
        for op in calls:
            tabs = []
            for segs in (op[1], op[2]):
                a = np.asarray(segs, dtype=np.int64).reshape(-1, 3)
                tabs.append((a[:, 0], a[:, 1], np.concatenate([[0], np.cumsum(a[:, 2])])))
            self.segs.append(tabs)

    def prefix(self, cid: int, src_ord: np.ndarray) -> np.ndarray:
        host, first, ob = self.segs[cid][0]
        k = np.searchsorted(ob[1:], src_ord, side="right")
        h = host[k]
        local = first[k] + (src_ord.astype(np.int64) - ob[k])
        a = int(self.calls[cid][5]) + 1
        return np.where(h == self.P_local, local, self.M_local + a * self.G + self.host_base[h] + local)

    def bucket(self, prefix: np.ndarray) -> np.ndarray:
        return ((prefix * NB) // self.pmax).astype(np.int16)

    def bucket_start(self, t: int) -> int:
        """first prefix of bucket t (t = NB: the end of the prefix space)"""
        return (t * self.pmax + NB - 1) // NB

    def local_ranges(self, cid: int, which: int, host: int):
        """ordinal ranges of the call's source (0) or target (1) set on `host`"""
        h, _, ob = self.segs[cid][which]
        return [(int(ob[k]), int(ob[k + 1])) for k in range(h.size) if h[k] == host and ob[k + 1] > ob[k]]


def work_items(layout: Layout, host: int = None, item_records: int = ITEM_RECORDS):
    """(call, lo, hi, cap) ranges of primary ordinals covering every call's
    share on `host` (default P_local)."""
    host = layout.P_local if host is None else host
    items = []
    for cid, op in enumerate(layout.calls):
        conn = op[3]
        rule = conn["rule"]
        ns = int(layout.segs[cid][0][2][-1])
        nt = int(layout.segs[cid][1][2][-1])
        if rule in ("fixed_indegree", "pairwise_bernoulli", "one_to_one"):
            per = {"fixed_indegree": int(conn.get("n", 0)), "one_to_one": 1}.get(rule, ns)
            if per == 0:
                continue
            step = max(1, item_records // per)
            for lo, hi in layout.local_ranges(cid, 1, host):
                for a in range(lo, hi, step):
                    b = min(hi, a + step)
                    items.append((cid, a, b, (b - a) * per))
        elif rule == "fixed_outdegree":
            K = int(conn.get("n", 0))
            if K == 0 or not layout.local_ranges(cid, 1, host):
                continue
            step = max(1, item_records // K)
            for a in range(0, ns, step):
                b = min(ns, a + step)
                items.append((cid, a, b, (b - a) * K))
        elif rule == "fixed_total_number":
            if int(conn.get("n", 0)) and layout.local_ranges(cid, 1, host):
                items.append((cid, 0, 2**63, int(conn["n"])))
        else:
            raise ValueError(f"rule {rule} not handled by the full-size harness")
    return items


# ---------------------------------------------------------------- worker side
_W = {}


def _init_worker(script: dict, P_local: int, call_ops: list, select_path: str | None):
    import oracle
    net = oracle.OracleNet(script["P"], P_local, script["seed"], script["dt"])
    for op in script["ops"]:
        if op[0] == "create":
            net.create(op[1], op[2])
    for op in call_ops:
        _, src, tgt, conn, syn, alpha = op
        net.declare(src, tgt, conn, syn, alpha)
    _W["net"] = net
    _W["layout"] = Layout(script, P_local, call_ops)
    _W["select"] = np.load(select_path, mmap_mode="r") if select_path else None


def _range(net, cid, host, lo, hi, cap):
    import oracle
    while True:
        try:
            return net.call_range(cid, host, lo, hi, max(1, cap))
        except oracle.OracleError:
            if cap >= 2**40:
                raise
            cap *= 4


def _phase_a(k: int, item, outdir: str, row_counts: bool):
    cid, lo, hi, cap = item
    L, net = _W["layout"], _W["net"]
    r = _range(net, cid, L.P_local, lo, hi, cap)
    pref = L.prefix(cid, r["src"])
    rows = None
    if row_counts:            # counts of every local source (one host, every source local)
        rows = np.bincount(pref, minlength=L.M_local).astype(np.int32)
    tgt, w, d = r["tgt"], r["weight"], r["delay"]
    sel = _W["select"]
    if sel is not None:
        keep = sel[pref]
        pref, tgt, w, d = pref[keep], tgt[keep], w[keep], d[keep]
    b = L.bucket(pref)
    order = np.argsort(b, kind="stable")
    counts = np.bincount(b, minlength=NB).astype(np.int64)
    off = np.concatenate([[0], np.cumsum(counts)])
    np.save(os.path.join(outdir, f"a{k}_p.npy"), pref[order])
    np.save(os.path.join(outdir, f"a{k}_t.npy"), tgt[order])
    np.save(os.path.join(outdir, f"a{k}_w.npy"), w[order])
    np.save(os.path.join(outdir, f"a{k}_d.npy"), d[order])
    np.save(os.path.join(outdir, f"a{k}_o.npy"), off)
    return k, int(r["src"].size), counts, rows


def _slices(outdir, items_k, t0, t1, names):
    out = {n: [] for n in names}
    for k in items_k:
        off = np.load(os.path.join(outdir, f"a{k}_o.npy"))
        a, b = int(off[t0]), int(off[t1])
        if a == b:
            continue
        for n in names:
            mm = np.load(os.path.join(outdir, f"a{k}_{n}.npy"), mmap_mode="r")
            out[n].append(np.array(mm[a:b]))      # a copy: the mapping (and its file) closes here
            del mm
    return {n: (np.concatenate(v) if v else None) for n, v in out.items()}


def _round_u(j: int, t0: int, t1: int, items_k, outdir: str):
    L = _W["layout"]
    s = _slices(outdir, items_k, t0, t1, ["p"])
    p = s["p"]
    u = np.unique(p[p >= L.M_local]) if p is not None else np.zeros(0, np.int64)
    np.save(os.path.join(outdir, f"u{j}.npy"), u)
    return j, int(u.size)


def _ulp(a: np.ndarray, b: np.ndarray) -> int:
    if a.size == 0:
        return 0
    ia = a.view(np.int32).astype(np.int64)
    ib = b.view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return int(np.abs(ia - ib).max())


def _phase_b(j: int, t0: int, t1: int, base: int, items_k, outdir: str, gpu_dir: str, s_lo: int, s_hi: int,
             rows_only: bool):
    """Sorted connections of source' range [s_lo, s_hi) against the library's.
    rows_only: the records are a selection of whole rows (compare those rows)."""
    L = _W["layout"]
    s = _slices(outdir, items_k, t0, t1, ["p", "t", "w", "d"])
    rp = np.load(os.path.join(gpu_dir, "row_ptr.npy"), mmap_mode="r")
    if s["p"] is None:
        if not rows_only and int(rp[s_hi]) != int(rp[s_lo]):
            return j, 0, f"source' [{s_lo}, {s_hi}): library has {int(rp[s_hi] - rp[s_lo])} connections, oracle none"
        return j, 0, None
    u = np.load(os.path.join(outdir, f"u{j}.npy"))
    p = s["p"]
    srcp = np.where(p < L.M_local, p, base + np.searchsorted(u, p))
    tbits = int(max(1, int(s["t"].max()) + 1)).bit_length()
    key = (srcp.astype(np.int64) << tbits) | s["t"].astype(np.int64)
    order = np.argsort(key, kind="stable")
    srcp, tgt, w, d = srcp[order], s["t"][order], s["w"][order], s["d"][order]
    n = srcp.size
    g = {name: np.load(os.path.join(gpu_dir, f"{name}.npy"), mmap_mode="r") for name in ("src", "tgt", "delay", "weight")}
    if rows_only:
        rows, starts = np.unique(srcp, return_index=True)
        ends = np.append(starts[1:], n)
        for r, a, b in zip(rows, starts, ends):
            ga, gb = int(rp[r]), int(rp[r + 1])
            if gb - ga != b - a:
                return j, n, f"row {r}: library {gb - ga} connections, oracle {b - a}"
            if not (np.array_equal(g["src"][ga:gb], srcp[a:b]) and np.array_equal(g["tgt"][ga:gb], tgt[a:b])
                    and np.array_equal(g["delay"][ga:gb], d[a:b])):
                return j, n, f"row {r} differs from the oracle"
            if _ulp(np.asarray(g["weight"][ga:gb]), w[a:b]) > 2:
                return j, n, f"row {r}: weights beyond 2 ulp"
        return j, n, None
    a, b = int(rp[s_lo]), int(rp[s_hi])
    if b - a != n:
        return j, n, f"source' [{s_lo}, {s_hi}): library {b - a} connections, oracle {n}"
    counts = np.bincount(srcp - s_lo, minlength=s_hi - s_lo)
    if not np.array_equal(np.diff(np.asarray(rp[s_lo:s_hi + 1], dtype=np.int64)), counts):
        return j, n, f"source' [{s_lo}, {s_hi}): row counts differ"
    for name, want in (("src", srcp), ("tgt", tgt), ("delay", d)):
        got = np.asarray(g[name][a:b])
        if not np.array_equal(got, want.astype(got.dtype)):
            i = int(np.flatnonzero(got != want.astype(got.dtype))[0])
            return j, n, f"{name}[{a + i}] = {got[i]}, oracle {want[i]} (source' range [{s_lo}, {s_hi}))"
    ulp = _ulp(np.asarray(g["weight"][a:b]), w)
    if ulp > 2:
        return j, n, f"weights {ulp} ulp from the oracle in source' [{s_lo}, {s_hi})"
    return j, n, None


def _send_list(cid: int, tau: int, lo: int, hi: int, cap: int):
    """local sources (on P_local) of tau's share of a call, sorted unique"""
    L, net = _W["layout"], _W["net"]
    r = _range(net, cid, tau, lo, hi, cap)
    host, first, ob = L.segs[cid][0]
    k = np.searchsorted(ob[1:], r["src"], side="right")
    on = host[k] == L.P_local
    local = first[k[on]] + (r["src"][on].astype(np.int64) - ob[k[on]])
    return tau, np.unique(local)


# ---------------------------------------------------------------- driver side
class FullSizeOracle:
    """The oracle's share of host P_local for the given (declared) calls,
    computed by `workers` processes into `workdir`."""

    def __init__(self, script: dict, P_local: int, call_ops: list, workdir: str, workers: int = 16,
                 select: np.ndarray | None = None, row_counts: bool = False, log=print,
                 item_records: int = ITEM_RECORDS, task_records: int = TASK_RECORDS):
        if (select is not None or row_counts) and script["P"] != 1:
            raise ValueError("row selections and row counts are for one-host networks (no images)")
        self.script, self.P_local, self.calls = script, P_local, call_ops
        self.item_records, self.task_records = item_records, task_records
        self.layout = Layout(script, P_local, call_ops)
        self.workdir = workdir
        self.log = log
        self.row_counts = row_counts
        os.makedirs(workdir, exist_ok=True)
        sel_path = None
        if select is not None:
            sel_path = os.path.join(workdir, "select.npy")
            np.save(sel_path, select.astype(bool))
        self.rows_only = select is not None
        small = {k: v for k, v in script.items() if k != "info"}
        self.pool = ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                                        initializer=_init_worker, initargs=(small, P_local, call_ops, sel_path))

    def close(self):
        self.pool.shutdown()

    # phase A and round U
    def generate(self):
        self.items = work_items(self.layout, item_records=self.item_records)
        futs = [self.pool.submit(_phase_a, k, it, self.workdir, self.row_counts) for k, it in enumerate(self.items)]
        self.counts = np.zeros(NB, np.int64)
        self.n_generated = 0
        self.rows = np.zeros(self.layout.M_local, np.int64) if self.row_counts else None
        import time
        from concurrent.futures import as_completed
        t_last = time.time()
        for done, f in enumerate(as_completed(futs), 1):
            k, n, counts, rows = f.result()
            self.counts += counts
            self.n_generated += n
            if rows is not None:
                self.rows += rows
            if time.time() - t_last > 20:
                self.log(f"oracle phase A: {done} of {len(futs)} items, {self.n_generated} connections")
                t_last = time.time()
        self.log(f"oracle: {len(self.items)} items, {self.n_generated} connections generated")
        # tasks: runs of buckets of about TASK_RECORDS records
        self.tasks, t0, acc = [], 0, 0
        for t in range(NB):
            acc += int(self.counts[t])
            if acc >= self.task_records or t == NB - 1:
                self.tasks.append((t0, t + 1))
                t0, acc = t + 1, 0
        ks = list(range(len(self.items)))
        res = list(self.pool.map(_round_u, range(len(self.tasks)), [a for a, _ in self.tasks],
                                 [b for _, b in self.tasks], [ks] * len(self.tasks), [self.workdir] * len(self.tasks)))
        sizes = np.array([n for _, n in sorted(res)], np.int64)
        self.task_base = self.layout.M_local + np.concatenate([[0], np.cumsum(sizes)])[:-1]
        self.U = np.concatenate([np.load(os.path.join(self.workdir, f"u{j}.npy")) for j in range(len(self.tasks))]) \
            if len(self.tasks) else np.zeros(0, np.int64)

    def src_prime(self, P: int) -> int:
        """source' of prefix P (first source' at or after it)"""
        if P <= self.layout.M_local:
            return P
        return self.layout.M_local + int(np.searchsorted(self.U, P))

    # maps
    def image_map(self) -> dict:
        L = self.layout
        n_slots = L.n_a * L.P
        starts = np.array([L.M_local + (k // L.P) * L.G + L.host_base[k % L.P] for k in range(n_slots)] +
                          [L.M_local + L.n_a * L.G], np.int64)
        r_off = np.searchsorted(self.U, starts).astype(np.uint64)
        slot = np.repeat(np.arange(n_slots), np.diff(r_off.astype(np.int64)))
        r_val = (self.U - starts[slot]).astype(np.int32)
        l_val = (L.M_local + np.arange(self.U.size)).astype(np.int32)
        img_base = (L.M_local + r_off[:-1].astype(np.int64)).astype(np.int64)
        return {"r_off": r_off, "r_val": r_val, "l_val": l_val, "img_base": img_base}

    # phase B
    def compare(self, gpu_dir: str):
        L = self.layout
        ks = list(range(len(self.items)))
        args = []
        for j, (t0, t1) in enumerate(self.tasks):
            s_lo = self.src_prime(L.bucket_start(t0))
            s_hi = self.src_prime(L.bucket_start(t1))
            args.append((j, t0, t1, int(self.task_base[j]), ks, self.workdir, gpu_dir, s_lo, s_hi, self.rows_only))
        import time
        from concurrent.futures import as_completed
        futs = [self.pool.submit(_phase_b, *a) for a in args]
        n, errors, t_last = 0, [], time.time()
        for done, f in enumerate(as_completed(futs), 1):
            j, m, err = f.result()
            n += m
            if err:
                errors.append(err)
            if time.time() - t_last > 20:
                self.log(f"oracle phase B: {done} of {len(futs)} tasks, {n} connections compared")
                t_last = time.time()
        return n, errors

    # point-to-point send lists of P_local
    def send_lists(self) -> dict:
        L = self.layout
        jobs = []
        for cid, op in enumerate(self.calls):
            if int(op[5]) != -1 or not L.local_ranges(cid, 0, L.P_local):
                continue
            K = int(op[3].get("n", 0))
            for tau in range(L.P):
                if tau == L.P_local:
                    continue
                for lo, hi in L.local_ranges(cid, 1, tau):
                    if op[3]["rule"] != "fixed_indegree":
                        raise ValueError("send lists of the harness cover fixed in-degree calls")
                    step = max(1, self.item_records // max(K, 1))
                    for a in range(lo, hi, step):
                        b = min(hi, a + step)
                        jobs.append((cid, tau, a, b, (b - a) * K))
        per_tau = {}
        for tau, s in self.pool.map(_send_list, *zip(*jobs)) if jobs else []:
            per_tau.setdefault(tau, []).append(s)
        S = [np.unique(np.concatenate(per_tau[t])) if t in per_tau else np.zeros(0, np.int64) for t in range(L.P)]
        s_off = np.concatenate([[0], np.cumsum([x.size for x in S])]).astype(np.uint64)
        s_val = np.concatenate(S).astype(np.int32) if S else np.zeros(0, np.int32)
        tau_of = np.repeat(np.arange(L.P), [x.size for x in S])
        pos_of = np.concatenate([np.arange(x.size) for x in S]) if S else np.zeros(0, np.int64)
        order = np.lexsort((tau_of, s_val))          # by source, then host ascending
        tp_ptr = np.concatenate([[0], np.cumsum(np.bincount(s_val, minlength=L.M_local))]).astype(np.uint64)
        return {"s_off": s_off, "s_val": s_val, "tp_ptr": tp_ptr, "t_val": tau_of[order].astype(np.uint32),
                "p_val": pos_of[order].astype(np.uint32)}

    # collective arrays of P_local
    def collective(self) -> dict:
        L = self.layout
        groups = sorted({int(op[5]) for op in self.calls if int(op[5]) >= 0})
        h_parts, i_parts, off = [], [], [0]
        gq = [[] for _ in range(L.M_local)] if L.M_local <= 5_000_000 else None
        for g_rank, alpha in enumerate(groups):
            for sigma in range(L.P):
                ids = [np.arange(f, f + n, dtype=np.int64) for op in self.calls if int(op[5]) == alpha
                       for h, f, n in op[1] if h == sigma and n]
                H = np.unique(np.concatenate(ids)) if ids else np.zeros(0, np.int64)
                if sigma == L.P_local:
                    I = np.full(H.size, -1, np.int64)
                    if gq is not None:
                        for pos, s in enumerate(H.tolist()):
                            gq[s].append((alpha, pos))
                else:
                    pre = L.M_local + (alpha + 1) * L.G + L.host_base[sigma] + H
                    at = np.searchsorted(self.U, pre)
                    hit = (at < self.U.size) & (self.U[np.minimum(at, max(self.U.size - 1, 0))] == pre) \
                        if self.U.size else np.zeros(H.size, bool)
                    I = np.where(hit, L.M_local + at, -1)
                h_parts.append(H)
                i_parts.append(I)
                off.append(off[-1] + H.size)
        out = {"groups": np.array(groups, np.int32), "h_off": np.array(off, np.uint64),
               "h_val": (np.concatenate(h_parts) if h_parts else np.zeros(0)).astype(np.int32),
               "i_val": (np.concatenate(i_parts) if i_parts else np.zeros(0)).astype(np.int32)}
        if gq is not None:
            out["gq_ptr"] = np.concatenate([[0], np.cumsum([len(x) for x in gq])]).astype(np.uint64)
            out["g_val"] = np.array([a for x in gq for a, _ in x], np.int32)
            out["q_val"] = np.array([q for x in gq for _, q in x], np.uint32)
        return out


def dump_library_arrays(net, gpu_dir: str, names=("src", "tgt", "delay", "weight", "row_ptr"), chunk=1 << 26):
    """Copy the library's prepared arrays into .npy files (memory-mapped by
    the workers)."""
    import paper_2512_09502_amd as snnc
    os.makedirs(gpu_dir, exist_ok=True)
    for name in names:
        n = net.count(name)
        dt = snnc.ARRAYS[name][1]
        out = np.lib.format.open_memmap(os.path.join(gpu_dir, f"{name}.npy"), mode="w+", dtype=dt, shape=(n,))
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            out[a:b] = net.array_range(name, a, b - a)
        out.flush()
        del out


# ---------------------------------------------------------------- served admission
def connect_ops(script):
    return [op for op in script["ops"] if op[0] == "connect"]


def meta_bytes(op, dt):
    """Resident metadata of a request, as the library documents it for
    snnc_set_resident_budget: 16 B per segment of each node set (at least
    one per set), 4 B per delay-table threshold plus a 257-word guide for a
    normal delay, 4 B for a constant one."""
    import oracle
    _, src, tgt, conn, syn, _ = op
    d = syn.get("delay") or {"kind": "const"}
    words = 1
    if d.get("kind") == "normal":
        tab = oracle.delay_table(d["mean"], d["sd"], d.get("lo", 0.0), dt)
        words = tab[1].size + 257 if tab is not None and tab[1].size else 1
    return 16 * (max(len(src), 1) + max(len(tgt), 1)) + 4 * words


def validate_requests(script):
    """Per request: 0 when valid (the oracle's validation), else its status;
    degrees above 8192 without multapses are unsupported (-5), the library's
    documented limit."""
    import oracle
    v = oracle.OracleNet(script["P"], 0, script["seed"], script["dt"])
    for op in script["ops"]:
        if op[0] == "create":
            v.create(op[1], op[2])
    status = []
    for op in connect_ops(script):
        _, src, tgt, conn, syn, alpha = op
        try:
            v.declare(src, tgt, conn, syn, alpha)
            big = conn["rule"] in ("fixed_indegree", "fixed_outdegree") and not conn.get("multapses", True) \
                and int(conn.get("n", 0)) > 8192
            status.append(-5 if big else 0)
        except oracle.OracleError as e:
            status.append(e.code)
    return status


def _expected(op):
    _, src, tgt, conn, _, _ = op
    ns, nt = sum(s[2] for s in src), sum(t[2] for t in tgt)
    r = conn["rule"]
    if r == "fixed_indegree":
        return nt * int(conn["n"])
    if r == "fixed_outdegree":
        return ns * int(conn["n"])
    if r == "fixed_total_number":
        return int(conn["n"])
    if r == "one_to_one":
        return ns
    return int(conn["p"] * ns * nt)


def _predict_ids(ops, status, meta, budget, counts):
    """call ids under the admission that the known counts give (expected
    counts for requests not yet counted with the id they would get)"""
    ids, resident, nxt = [None] * len(ops), 0, 0
    for k, op in enumerate(ops):
        if status[k] != 0:
            continue
        n = counts.get((k, nxt))
        if n is None:
            n = _expected(op)
        ids[k] = nxt
        if resident + 14 * n + meta[k] <= budget:
            resident += 14 * n + meta[k]
            nxt += 1
    return ids


def _count_jobs(op, k, cid, pairs_per_job=200_000_000):
    _, src, tgt, conn, _, _ = op
    if conn["rule"] != "pairwise_bernoulli":
        return [(op, k, cid, 0, 2**63)]
    ns, nt = sum(s[2] for s in src), sum(t[2] for t in tgt)
    step = max(1, pairs_per_job // max(ns, 1))
    return [(op, k, cid, a, min(nt, a + step)) for a in range(0, nt, step)]


def _count_job(script, job):
    """count of request k under call id cid (primary ordinals [lo, hi)):
    cid placeholder calls are declared first, so the request gets that id"""
    import oracle
    op, k, cid, lo, hi = job
    net = oracle.OracleNet(script["P"], 0, script["seed"], script["dt"])
    first = None
    for o in script["ops"]:
        if o[0] == "create":
            seg = net.create(o[1], o[2])
            first = first or seg
    one = [(first[0], first[1], 1)]
    for _ in range(cid):
        net.declare(one, one, {"rule": "one_to_one"}, {"weight": {"kind": "const", "mean": 0.0},
                                                        "delay": {"kind": "const", "mean": 1.0}})
    _, src, tgt, conn, syn, alpha = op
    got = net.declare(src, tgt, conn, syn, alpha)
    assert got == cid
    return (k, cid), net.call_count(cid, 0, lo, hi)


def served_admission(script, budget: int, workers: int = 16, pairs_per_job: int = 200_000_000):
    """The oracle's admission of a one-host request stream against a resident
    budget: requests in order; a valid request is admitted when the resident
    bytes plus 14 B per connection of its count plus its metadata fit the
    budget, and then gets the next call id.  A count depends on the call id
    (the draws are keyed by it), so counts are computed in parallel for the
    ids a prediction gives and computed again for any request whose id turns
    out different; the result is the sequential admission.  Returns the
    status per request (0, -3 over budget, or the validation status), the
    admitted request indices and their counts."""
    ops = connect_ops(script)
    status = validate_requests(script)
    meta = [meta_bytes(op, script["dt"]) for op in ops]
    small = {k: v for k, v in script.items() if k != "info"}
    counts = {}
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as pool:
        ids = _predict_ids(ops, status, meta, budget, counts)
        for _ in range(50):
            todo = [k for k in range(len(ops)) if status[k] == 0 and (k, ids[k]) not in counts]
            if not todo:
                break
            jobs = [j for k in todo for j in _count_jobs(ops[k], k, ids[k], pairs_per_job)]
            partial = {}
            for key, n in pool.map(_count_job, [small] * len(jobs), jobs, chunksize=1):
                partial[key] = partial.get(key, 0) + n
            counts.update(partial)
            ids = _predict_ids(ops, status, meta, budget, counts)
        else:
            raise RuntimeError("served admission did not settle")
    admitted, count_of, resident = [], [], 0
    status = list(status)
    for k in range(len(ops)):
        if status[k] != 0:
            continue
        n = counts[(k, len(admitted))]
        if resident + 14 * n + meta[k] <= budget:
            resident += 14 * n + meta[k]
            admitted.append(k)
            count_of.append(n)
        else:
            status[k] = -3
    return status, admitted, count_of
