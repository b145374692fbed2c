"""CPU oracle for on-device spiking-network construction -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``snnc_oracle.c`` (plain,
single-threaded C; see the header of that file for what it computes and which
passages of arXiv:2512.09502 each step follows) through ctypes.  It shares no
code with the GPU library and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "snnc_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

RULES = {"one_to_one": 0, "fixed_indegree": 1, "fixed_outdegree": 2,
         "fixed_total_number": 3, "pairwise_bernoulli": 4, "assigned_nodes": 5}
DISTS = {"const": 0, "normal": 1}

# array ids and dtypes (same numbering as the C file's accessor enum)
ARRAYS = {
    "gen_src": (0, np.uint32), "gen_tgt": (1, np.uint32), "gen_delay": (2, np.uint16),
    "gen_weight": (3, np.float32), "gen_e": (4, np.uint64), "call_off": (5, np.uint64),
    "src": (10, np.int32), "tgt": (11, np.int32), "delay": (12, np.uint16),
    "weight": (13, np.float32), "row_ptr": (14, np.uint64),
    "img_first": (15, np.uint64), "img_count": (16, np.uint32),
    "r_off": (20, np.uint64), "r_val": (21, np.int32), "img_base": (22, np.int64),
    "l_val": (23, np.int32),
    "s_off": (30, np.uint64), "s_val": (31, np.int32), "tp_ptr": (32, np.uint64),
    "t_val": (33, np.uint32), "p_val": (34, np.uint32),
    "groups": (40, np.int32), "h_off": (41, np.uint64), "h_val": (42, np.int32),
    "i_val": (43, np.int32), "gq_ptr": (44, np.uint64), "g_val": (45, np.int32),
    "q_val": (46, np.uint32),
}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u32, u64, i32, i64, dbl = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                                   ctypes.c_int64, ctypes.c_double)
        vp = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_uniform_index.argtypes = [u32, u32, u64]
        L.orc_uniform_index.restype = u64
        L.orc_normal_weight.argtypes = [u32, u32, dbl, dbl]
        L.orc_normal_weight.restype = ctypes.c_float
        L.orc_delay_table.argtypes = [dbl, dbl, dbl, dbl, vp, u64, vp]
        L.orc_delay_table.restype = i64
        L.orc_new.argtypes = [u32, u32, u32, dbl]
        L.orc_new.restype = vp
        L.orc_free.argtypes = [vp]
        L.orc_last_error.argtypes = [vp]
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_create.argtypes = [vp, u32, u32, vp]
        conn_args = [vp, vp, u32, vp, u32, ctypes.c_int, u64, dbl, ctypes.c_int, ctypes.c_int,
                     ctypes.c_int, dbl, dbl, ctypes.c_int, dbl, dbl, dbl, i32, vp]
        L.orc_connect.argtypes = conn_args
        L.orc_declare.argtypes = conn_args
        L.orc_call_count.argtypes = [vp, u32, u32, u64, u64]
        L.orc_call_count.restype = i64
        L.orc_connect_assigned.argtypes = [vp, vp, u32, vp, u32, vp, vp, u64,
                                           ctypes.c_int, dbl, dbl, ctypes.c_int, dbl, dbl, dbl, i32, vp]
        L.orc_prepare.argtypes = [vp]
        L.orc_set_map_policy.argtypes = [vp, ctypes.c_int, ctypes.c_int, dbl]
        L.orc_set_memory_level.argtypes = [vp, ctypes.c_int]
        L.orc_packets_from_lists.restype = ctypes.c_int64
        L.orc_packets_from_lists.argtypes = [vp, vp, vp, u32, u32, vp, vp, u64, vp, vp, vp, u64]
        L.orc_spike_packets.restype = ctypes.c_int64
        L.orc_spike_packets.argtypes = [vp, ctypes.c_int, vp, vp, u64, vp, vp, vp, u64]
        L.orc_deliver_from_maps.restype = ctypes.c_int64
        L.orc_deliver_from_maps.argtypes = [vp, vp, u64, vp, vp, vp, vp, vp, vp, vp, u64, vp, vp, vp, vp, vp, vp, u64]
        L.orc_deliver.restype = ctypes.c_int64
        L.orc_deliver.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, u64, vp, vp, vp, vp, vp, vp, u64]
        L.orc_len.argtypes = [vp, ctypes.c_int]
        L.orc_len.restype = i64
        L.orc_copy.argtypes = [vp, ctypes.c_int, vp, u64]
        L.orc_neurons.argtypes = [vp, u32]
        L.orc_neurons.restype = u32
        L.orc_call_range.argtypes = [vp, u32, u32, u64, u64, vp, vp, vp, vp, vp, u64]
        L.orc_call_range.restype = i64
        L.orc_call_element.argtypes = [vp, u32, u64, vp, vp, vp, vp, vp]
        L.orc_call_element.restype = ctypes.c_int
        L.orc_sort_csr.argtypes = [u64, vp, vp, vp, vp, u64, vp, vp, vp, vp, vp]
        L.orc_transpose_lists.argtypes = [u32, vp, vp, u32, vp, vp, vp]
        L.orc_transpose_lists.restype = u64
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- primitives
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform_index(lo: int, hi: int, n: int) -> int:
    return int(lib().orc_uniform_index(lo, hi, n))


def normal_weight(w0: int, w1: int, mean: float, sd: float) -> float:
    return float(lib().orc_normal_weight(w0, w1, mean, sd))


def delay_table(mean: float, sd: float, lo: float, dt: float):
    """Return (k_lo, thresholds uint32[]) or None if it does not fit."""
    buf = np.zeros(65536, np.uint32)
    klo = np.zeros(1, np.uint32)
    n = lib().orc_delay_table(mean, sd, lo, dt, _ptr(buf), buf.size, _ptr(klo))
    if n < 0:
        return None
    return int(klo[0]), buf[:n].copy()


def sort_csr(src, tgt, delay, weight, n_rows: int) -> dict:
    """The source-major sort and first-index step on given arrays."""
    src = np.ascontiguousarray(src, np.int32)
    tgt = np.ascontiguousarray(tgt, np.uint32)
    delay = np.ascontiguousarray(delay, np.uint16)
    weight = np.ascontiguousarray(weight, np.float32)
    n = src.size
    out = {"src": np.zeros(n, np.int32), "tgt": np.zeros(n, np.int32),
           "delay": np.zeros(n, np.uint16), "weight": np.zeros(n, np.float32),
           "row_ptr": np.zeros(n_rows + 1, np.uint64)}
    lib().orc_sort_csr(n, _ptr(src), _ptr(tgt), _ptr(delay), _ptr(weight), n_rows,
                       _ptr(out["src"]), _ptr(out["tgt"]), _ptr(out["delay"]), _ptr(out["weight"]),
                       _ptr(out["row_ptr"]))
    return out


def transpose_lists(lists, M: int):
    """Per-neuron (list index, position) pairs of sorted lists (T/P, G/Q)."""
    off = np.zeros(len(lists) + 1, np.uint64)
    for k, l in enumerate(lists):
        off[k + 1] = off[k] + len(l)
    val = np.ascontiguousarray(np.concatenate([np.asarray(l, np.int32) for l in lists])
                               if lists else np.zeros(0, np.int32), np.int32)
    ptr = np.zeros(M + 1, np.uint64)
    cap = max(1, int(off[-1]))
    which = np.zeros(cap, np.uint32)
    pos = np.zeros(cap, np.uint32)
    n = lib().orc_transpose_lists(len(lists), _ptr(off), _ptr(val), M, _ptr(ptr), _ptr(which), _ptr(pos))
    return ptr, which[:n], pos[:n]


def _u32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def _packets_result(r, off, pos, mult):
    if r < 0:
        raise OracleError(-1, "spike id out of range")
    return {"off": off, "pos": pos[:r], "mult": mult[:r]}


def packets_from_lists(ptr, dest, where, M: int, n_dest: int, spikes, mult=None) -> dict:
    """Packets of one step from explicit per-source lists (Appendix E)."""
    ptr = np.ascontiguousarray(np.asarray(ptr, dtype=np.uint64))
    dest, where, spikes = _u32(dest), _u32(where), _u32(spikes)
    mult = None if mult is None else _u32(mult)
    ok = spikes[spikes < ptr.size - 1].astype(np.int64)
    cap = int((ptr[ok + 1].astype(np.int64) - ptr[ok].astype(np.int64)).sum())
    off = np.zeros(n_dest + 1, np.uint64)
    pos, mo = np.zeros(max(cap, 1), np.uint32), np.zeros(max(cap, 1), np.uint32)
    r = lib().orc_packets_from_lists(_ptr(ptr), _ptr(dest), _ptr(where), M, n_dest, _ptr(spikes),
                                     None if mult is None else _ptr(mult), len(spikes), _ptr(off), _ptr(pos),
                                     _ptr(mo), cap)
    return _packets_result(r, off, pos, mo)


def _deliver_result(r, image, rb, re, et, ed, ew):
    if r == -1:
        raise OracleError(-1, "entry outside its map")
    return {"image": image, "row_begin": rb, "row_end": re, "tgt": et[:r], "delay": ed[:r], "weight": ew[:r]}


def deliver_from_maps(map_off, map_img, row_ptr, tgt, delay, weight, key, pos, mult=None) -> dict:
    """Delivery through explicit maps and sorted connection arrays (Appendix E)."""
    map_off = np.ascontiguousarray(np.asarray(map_off, dtype=np.uint64))
    map_img = np.ascontiguousarray(np.asarray(map_img, dtype=np.int32))
    row_ptr = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.uint64))
    tgt = np.ascontiguousarray(np.asarray(tgt, dtype=np.int32))
    delay = np.ascontiguousarray(np.asarray(delay, dtype=np.uint16))
    weight = np.ascontiguousarray(np.asarray(weight, dtype=np.float32))
    key, pos = _u32(key), _u32(pos)
    mult = None if mult is None else _u32(mult)
    n = len(key)
    image, rb, re = np.zeros(max(n, 1), np.int32), np.zeros(max(n, 1), np.uint64), np.zeros(max(n, 1), np.uint64)
    args = (_ptr(map_off), _ptr(map_img), map_off.size - 1, _ptr(row_ptr), _ptr(tgt), _ptr(delay), _ptr(weight),
            _ptr(key), _ptr(pos), None if mult is None else _ptr(mult), n, _ptr(image), _ptr(rb), _ptr(re))
    cap = lib().orc_deliver_from_maps(*args, None, None, None, 0)   # event count first
    if cap < 0:
        return _deliver_result(cap, image, rb, re, None, None, None)
    et, ed, ew = np.zeros(max(cap, 1), np.int32), np.zeros(max(cap, 1), np.uint16), np.zeros(max(cap, 1), np.float32)
    r = lib().orc_deliver_from_maps(*args, _ptr(et), _ptr(ed), _ptr(ew), cap)
    return _deliver_result(r, image[:n], rb[:n], re[:n], et, ed, ew)


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


# ---------------------------------------------------------------- network
def _triples(segs) -> np.ndarray:
    a = np.asarray(segs, dtype=np.uint32).reshape(-1, 3)
    return np.ascontiguousarray(a)


def _dist(d):
    if d is None:
        return 0, 0.0, 0.0, 0.0
    kind = DISTS[d.get("kind", "const")]
    return kind, float(d.get("mean", 0.0)), float(d.get("sd", 0.0)), float(d.get("lo", 0.0))


class OracleNet:
    """One host's share of a network, built by the C oracle."""

    def __init__(self, P: int, P_local: int, seed: int, dt: float):
        self._h = lib().orc_new(P, P_local, seed, dt)
        if not self._h:
            raise OracleError(-1, "invalid P/P_local/dt")
        self.P, self.P_local = P, P_local

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    def _check(self, st):
        if st != 0:
            raise OracleError(st, lib().orc_last_error(self._h).decode())

    def create(self, host: int, n: int) -> tuple:
        first = np.zeros(1, np.uint32)
        self._check(lib().orc_create(self._h, host, n, _ptr(first)))
        return (host, int(first[0]), n)

    def _conn(self, fn, src, tgt, conn, syn, alpha):
        s, t = _triples(src), _triples(tgt)
        wk, wm, wsd, _ = _dist(syn.get("weight"))
        dk, dm, dsd, dlo = _dist(syn.get("delay"))
        cid = np.zeros(1, np.uint32)
        st = fn(self._h, _ptr(s), s.shape[0], _ptr(t), t.shape[0], RULES[conn["rule"]],
                int(conn.get("n", 0)), float(conn.get("p", 0.0)),
                int(conn.get("autapses", True)), int(conn.get("multapses", True)),
                wk, wm, wsd, dk, dm, dsd, dlo, int(alpha), _ptr(cid))
        self._check(st)
        return int(cid[0])

    def connect(self, src, tgt, conn, syn, alpha=-1) -> int:
        if conn["rule"] == "assigned_nodes":
            return self._assigned(src, tgt, conn, syn, alpha)
        return self._conn(lib().orc_connect, src, tgt, conn, syn, alpha)

    def _assigned(self, src, tgt, conn, syn, alpha):
        """Assigned nodes: conn["pairs"] = (source positions, target positions)."""
        s, t = _triples(src), _triples(tgt)
        ps = np.ascontiguousarray(conn["pairs"][0], dtype=np.uint32)
        pt = np.ascontiguousarray(conn["pairs"][1], dtype=np.uint32)
        if ps.shape != pt.shape:
            raise OracleError(-1, "pair arrays differ in length")
        wk, wm, wsd, _ = _dist(syn.get("weight"))
        dk, dm, dsd, dlo = _dist(syn.get("delay"))
        cid = np.zeros(1, np.uint32)
        st = lib().orc_connect_assigned(self._h, _ptr(s), s.shape[0], _ptr(t), t.shape[0], _ptr(ps), _ptr(pt),
                                        ps.size, wk, wm, wsd, dk, dm, dsd, dlo, int(alpha), _ptr(cid))
        self._check(st)
        return int(cid[0])

    def declare(self, src, tgt, conn, syn, alpha=-1) -> int:
        return self._conn(lib().orc_declare, src, tgt, conn, syn, alpha)

    def set_map_policy(self, numbering: int, sources: int, xi: float = 1.0):
        """numbering: 0 canonical, 1 in call order; sources: 0 used,
        1 threshold heuristic with xi, 2 all passed sources."""
        self._check(lib().orc_set_map_policy(self._h, int(numbering), int(sources), float(xi)))

    def set_memory_level(self, level: int):
        """GPU memory level 0..3: images of used (0) or all passed sources
        (1..3), and which image-row arrays exist."""
        self._check(lib().orc_set_memory_level(self._h, int(level)))

    def prepare(self):
        self._check(lib().orc_prepare(self._h))

    def neurons(self, host: int) -> int:
        return int(lib().orc_neurons(self._h, host))

    def array(self, name: str) -> np.ndarray:
        which, dt = ARRAYS[name]
        n = lib().orc_len(self._h, which)
        if n < 0:
            raise OracleError(-4, f"array {name} not available")
        out = np.zeros(n, dt)
        self._check(lib().orc_copy(self._h, which, _ptr(out), out.nbytes))
        return out

    def element(self, call_id: int, e: int):
        """One element of a call computed on its own: None if it is not a
        connection; raises for rules whose elements depend on each other."""
        so, th, tl = (ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32())
        w, d = ctypes.c_float(), ctypes.c_uint16()
        r = lib().orc_call_element(self._h, call_id, e, ctypes.byref(so), ctypes.byref(th), ctypes.byref(tl),
                                   ctypes.byref(w), ctypes.byref(d))
        if r < 0:
            raise OracleError(-1, "element not computable on its own for this call")
        if r == 0:
            return None
        return {"src": so.value, "tgt_host": th.value, "tgt": tl.value, "weight": w.value, "delay": d.value}

    def spike_packets(self, kind: int, spikes, mult=None) -> dict:
        """Packets of one step: kind 0 per target host (T/P), kind 1 per group (G/Q)."""
        spikes = _u32(spikes)
        mult = None if mult is None else _u32(mult)
        n_dest = self.P if kind == 0 else len(self.array("groups"))
        ptr = self.array("tp_ptr" if kind == 0 else "gq_ptr").astype(np.int64)
        ok = spikes[spikes < ptr.size - 1].astype(np.int64)
        cap = max(1, int((ptr[ok + 1] - ptr[ok]).sum()))
        off = np.zeros(n_dest + 1, np.uint64)
        pos, mo = np.zeros(cap, np.uint32), np.zeros(cap, np.uint32)
        r = lib().orc_spike_packets(self._h, kind, _ptr(spikes), None if mult is None else _ptr(mult), len(spikes),
                                    _ptr(off), _ptr(pos), _ptr(mo), cap)
        return _packets_result(r, off, pos, mo)

    def deliver(self, kind: int, host, pos, mult=None, grp=None) -> dict:
        """Delivery of received entries: kind 0 (sigma, i) through L, kind 1
        (group rank, sigma, j) through I; per entry image and row, and events."""
        host, pos = _u32(host), _u32(pos)
        grp = None if grp is None else _u32(grp)
        mult = None if mult is None else _u32(mult)
        n = len(host)
        image, rb, re = np.zeros(max(n, 1), np.int32), np.zeros(max(n, 1), np.uint64), np.zeros(max(n, 1), np.uint64)
        args = (self._h, kind, None if grp is None else _ptr(grp), _ptr(host), _ptr(pos),
                None if mult is None else _ptr(mult), n, _ptr(image), _ptr(rb), _ptr(re))
        cap = lib().orc_deliver(*args, None, None, None, 0)          # event count first
        if cap < 0:
            return _deliver_result(cap, image, rb, re, None, None, None)
        et, ed, ew = np.zeros(max(cap, 1), np.int32), np.zeros(max(cap, 1), np.uint16), np.zeros(max(cap, 1), np.float32)
        r = lib().orc_deliver(*args, _ptr(et), _ptr(ed), _ptr(ew), cap)
        return _deliver_result(r, image[:n], rb[:n], re[:n], et, ed, ew)

    def call_range(self, call_id: int, host: int, lo: int, hi: int, cap: int) -> dict:
        """Draws of one call on one host's share, primary ordinal in [lo, hi)."""
        src = np.zeros(cap, np.uint32)
        tgt = np.zeros(cap, np.uint32)
        e = np.zeros(cap, np.uint64)
        w = np.zeros(cap, np.float32)
        d = np.zeros(cap, np.uint16)
        n = lib().orc_call_range(self._h, call_id, host, lo, hi, _ptr(src), _ptr(tgt), _ptr(e),
                                 _ptr(w), _ptr(d), cap)
        if n < 0:
            raise OracleError(-1, "call_range: capacity too small or bad call id")
        return {"src": src[:n], "tgt": tgt[:n], "e": e[:n], "weight": w[:n], "delay": d[:n]}

    def call_count(self, call_id: int, host: int, lo: int = 0, hi: int = 2**63) -> int:
        """Connections of a call on one host's share (primary ordinal in [lo,
        hi)), counted by the same walk of the draws as the generation."""
        n = lib().orc_call_count(self._h, call_id, host, lo, hi)
        if n < 0:
            raise OracleError(-1, "call_count: bad call id")
        return int(n)


def run_script(script, P_local: int, declare_only: bool = False, skip_invalid: bool = False):
    """Replay a workload script (see ``paper_2512_09502_amd.workloads``) on host
    P_local.  With ``skip_invalid`` a rejected connect is recorded in
    ``net.rejected`` as (op index, status) and the replay goes on."""
    net = OracleNet(script["P"], P_local, script["seed"], script["dt"])
    if script.get("memory_level") is not None:
        net.set_memory_level(script["memory_level"])
    if script.get("map_policy") is not None:
        net.set_map_policy(*script["map_policy"])
    net.rejected = []
    for k, op in enumerate(script["ops"]):
        if op[0] == "create":
            net.create(op[1], op[2])
            continue
        _, src, tgt, conn, syn, alpha = op
        try:
            if declare_only:
                net.declare(src, tgt, conn, syn, alpha)
            else:
                net.connect(src, tgt, conn, syn, alpha)
        except OracleError as err:
            if not skip_invalid:
                raise
            net.rejected.append((k, err.code))
    if not declare_only:
        net.prepare()
    return net
