"""MI355X (gfx950) spiking-network construction: Python binding of libsnnc.

A thin ctypes layer over the C ABI declared in ``include/snnc.h``: it only
marshals arguments.  Every step of the construction runs in the HIP library;
there is no CPU fallback -- if ``libsnnc.so`` is missing or no GPU is
visible, the calls raise.  PyTorch provides device memory (its caching
allocator, through the library's allocator callbacks) and the HIP stream.
"""
from __future__ import annotations

import ctypes
import os
import struct

import numpy as np

from . import workloads  # noqa: F401  (seeded workload scripts)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnnc.so")

RULES = {"one_to_one": 0, "fixed_indegree": 1, "fixed_outdegree": 2,
         "fixed_total_number": 3, "pairwise_bernoulli": 4, "assigned_nodes": 5}
DISTS = {"const": 0, "normal": 1}
STATUS = {0: "SNNC_OK", -1: "SNNC_EINVAL", -2: "SNNC_ENOMEM", -3: "SNNC_EBUDGET",
          -4: "SNNC_ESTATE", -5: "SNNC_EUNSUPPORTED", -6: "SNNC_EDEVICE"}

# array name -> (snnc_array_id, numpy dtype)
ARRAYS = {
    "gen_src": (0, np.uint32), "gen_tgt": (1, np.uint32), "gen_delay": (2, np.uint16),
    "gen_weight": (3, np.float32), "call_off": (5, np.uint64),
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


class Segment(ctypes.Structure):
    _fields_ = [("host", ctypes.c_uint32), ("first", ctypes.c_uint32), ("n", ctypes.c_uint32)]


class NodeSet(ctypes.Structure):
    _fields_ = [("seg", ctypes.POINTER(Segment)), ("n_seg", ctypes.c_uint32)]


class ConnSpec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("allow_autapses", ctypes.c_uint32),
                ("allow_multapses", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("n", ctypes.c_uint64), ("p", ctypes.c_double)]


class Dist(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("mean", ctypes.c_double), ("sd", ctypes.c_double), ("lo", ctypes.c_double)]


class SynSpec(ctypes.Structure):
    _fields_ = [("weight", Dist), ("delay_ms", Dist), ("port", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("n_connections", ctypes.c_uint64), ("n_images", ctypes.c_uint64),
                ("n_calls", ctypes.c_uint32), ("M_local", ctypes.c_uint32),
                ("bytes_live", ctypes.c_uint64), ("bytes_peak", ctypes.c_uint64),
                ("sort_passes", ctypes.c_uint32), ("key_bits", ctypes.c_uint32),
                ("ms_connect", ctypes.c_double), ("ms_prepare", ctypes.c_double)]


EXPORTS = ["snnc_init", "snnc_destroy", "snnc_last_error", "snnc_sync", "snnc_create", "snnc_connect",
           "snnc_reserve", "snnc_prepare", "snnc_get_array", "snnc_copy_array", "snnc_copy_range",
           "snnc_stats", "snnc_set_timing", "snnc_kernel_times", "snnc_delay_table", "snnc_philox_blocks",
           "snnc_tune", "snnc_sort_pairs", "snnc_set_resident_budget", "snnc_submit", "snnc_submit_many", "snnc_flush", "snnc_poll",
           "snnc_autotune_sort", "snnc_set_map_policy", "snnc_spike_packets", "snnc_deliver",
           "snnc_connect_assigned", "snnc_set_memory_level", "snnc_array_on_host", "snnc_get_connections",
           "snnc_get_image_map", "snnc_get_p2p_send", "snnc_get_collective", "snnc_copy_to_host",
           "snnc_sort_pairs_noalloc", "snnc_autotune_fused"]

_lib = None


_P = ctypes.c_void_p
_U64, _U32, _I32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32


class ConnView(ctypes.Structure):
    _fields_ = [("src", _P), ("tgt", _P), ("delay", _P), ("weight", _P), ("row_ptr", _P), ("img_first", _P),
                ("img_count", _P), ("n", _U64), ("n_rows", _U64), ("n_images", _U64), ("M_local", _U32),
                ("img_rows_on_host", _I32)]


class P2PView(ctypes.Structure):
    _fields_ = [("s_off", _P), ("s_val", _P), ("tp_ptr", _P), ("t_val", _P), ("p_val", _P), ("n_s", _U64),
                ("n_tp", _U64), ("P", _U32), ("M_local", _U32)]


class CollView(ctypes.Structure):
    _fields_ = [("h_off", _P), ("h_val", _P), ("i_val", _P), ("gq_ptr", _P), ("g_val", _P), ("q_val", _P),
                ("n_h", _U64), ("n_gq", _U64), ("alpha", _I32), ("rank", _U32), ("P", _U32), ("M_local", _U32),
                ("on_host", _I32)]

def lib():
    """Load libsnnc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2512_09502_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32, dbl = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        st = ctypes.c_int
        L.snnc_init.argtypes = [ctypes.POINTER(vp), u32, u32, u32, dbl, ctypes.POINTER(Allocator), vp, u64]
        L.snnc_destroy.argtypes = [vp]
        L.snnc_last_error.argtypes = [vp]
        L.snnc_last_error.restype = ctypes.c_char_p
        L.snnc_sync.argtypes = [vp]
        L.snnc_create.argtypes = [vp, u32, u32, ctypes.POINTER(Segment)]
        L.snnc_connect.argtypes = [vp, ctypes.POINTER(NodeSet), ctypes.POINTER(NodeSet), ctypes.POINTER(ConnSpec),
                                   ctypes.POINTER(SynSpec), i32, ctypes.POINTER(u32)]
        L.snnc_reserve.argtypes = [vp, u64]
        L.snnc_prepare.argtypes = [vp]
        L.snnc_set_map_policy.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double]
        L.snnc_set_memory_level.argtypes = [vp, ctypes.c_int32]
        L.snnc_array_on_host.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32)]
        L.snnc_spike_packets.argtypes = [vp, ctypes.c_int32, vp, vp, u64, vp, vp, vp, u64, ctypes.POINTER(u64)]
        L.snnc_deliver.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, u64, vp, vp, vp, vp, vp, vp, u64,
                                   ctypes.POINTER(u64)]
        L.snnc_get_array.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(u64)]
        L.snnc_copy_array.argtypes = [vp, i32, vp, u64]
        L.snnc_copy_range.argtypes = [vp, i32, u64, u64, vp]
        L.snnc_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.snnc_set_timing.argtypes = [vp, ctypes.c_int]
        L.snnc_kernel_times.argtypes = [vp, u32, vp, vp, vp, ctypes.POINTER(u32)]
        L.snnc_delay_table.argtypes = [dbl, dbl, dbl, dbl, vp, u64, ctypes.POINTER(u32), ctypes.POINTER(u64)]
        L.snnc_philox_blocks.argtypes = [vp, u32, u32, u64, u32, u64, vp]
        L.snnc_tune.argtypes = [vp, ctypes.c_char_p, ctypes.c_int64]
        L.snnc_sort_pairs.argtypes = [vp, vp, vp, vp, vp, u64, u32, u32, ctypes.POINTER(ctypes.c_int32)]
        L.snnc_sort_pairs_noalloc.argtypes = L.snnc_sort_pairs.argtypes
        L.snnc_autotune_fused.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float)]
        L.snnc_set_resident_budget.argtypes = [vp, u64]
        L.snnc_submit.argtypes = L.snnc_connect.argtypes
        L.snnc_connect_assigned.argtypes = [vp, ctypes.POINTER(NodeSet), ctypes.POINTER(NodeSet), vp, vp, u64,
                                            ctypes.POINTER(SynSpec), i32, ctypes.POINTER(u32)]
        L.snnc_submit_many.argtypes = [vp, u32, vp, vp, vp, vp, vp, vp, vp]
        L.snnc_flush.argtypes = [vp]
        L.snnc_poll.argtypes = [vp, u32, ctypes.POINTER(ctypes.c_int32)]
        L.snnc_autotune_sort.argtypes = [vp, u64, u32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_float)]
        L.snnc_get_connections.argtypes = [vp, ctypes.POINTER(ConnView)]
        L.snnc_get_image_map.argtypes = [vp, i32, u32, ctypes.POINTER(vp), ctypes.POINTER(u64),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(vp)]
        L.snnc_get_p2p_send.argtypes = [vp, ctypes.POINTER(P2PView)]
        L.snnc_get_collective.argtypes = [vp, i32, ctypes.POINTER(CollView)]
        L.snnc_copy_to_host.argtypes = [vp, i32, vp, u64]
        for name in EXPORTS:
            getattr(L, name).restype = st if name != "snnc_last_error" else ctypes.c_char_p
        # connect and submit with their structs passed as plain addresses into
        # one packed buffer (see Network._connect_like)
        proto = ctypes.CFUNCTYPE(st, vp, ctypes.c_size_t, ctypes.c_size_t, ctypes.c_size_t, ctypes.c_size_t, i32,
                                 ctypes.c_size_t)
        L.packed = {name: proto((name, L)) for name in ("snnc_connect", "snnc_submit")}
        _lib = L
    return _lib


class SnncError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _dist(d) -> Dist:
    d = d or {"kind": "const", "mean": 0.0}
    return Dist(DISTS[d.get("kind", "const")], 0, float(d.get("mean", 0.0)), float(d.get("sd", 0.0)),
                float(d.get("lo", 0.0)))


# Packed connect arguments, C layout without padding: snnc_conn_spec (32 B),
# snnc_syn_spec (72 B), source and target snnc_nodeset (16 B each), the call
# id (4 B, then 4 B pad), then the segments (12 B each).
_SPEC = struct.Struct("<IIIIQdIIdddIIdddII")
_NODESETS = struct.Struct("<QI4xQI4x")
_OFF_SYN, _OFF_NS, _OFF_CID, _OFF_SEG = 32, 104, 136, 144
_SEGS = {}
_CONST0 = {"kind": "const", "mean": 0.0}


def _seg_struct(n):
    f = _SEGS.get(n)
    if f is None:
        f = _SEGS[n] = struct.Struct("<" + "III" * n)
    return f


def _nodeset(segs):
    arr = (Segment * max(1, len(segs)))(*[Segment(int(h), int(f), int(n)) for h, f, n in segs])
    return NodeSet(arr, len(segs)), arr


def delay_table(mean: float, sd: float, lo: float, dt: float):
    """The library's host-built delay table: (k_lo, thresholds) or None."""
    buf = np.zeros(65536, np.uint32)
    klo = ctypes.c_uint32()
    n = ctypes.c_uint64()
    st = lib().snnc_delay_table(mean, sd, lo, dt, buf.ctypes.data, buf.size, ctypes.byref(klo), ctypes.byref(n))
    if st != 0:
        return None
    return int(klo.value), buf[: n.value].copy()


class RequestBatch:
    """Connect requests marshalled once into the C structs of the ABI
    (snnc_nodeset, snnc_conn_spec, snnc_syn_spec and alpha arrays; segments
    in one array), so that snnc_submit_many or snnc_connect can take any
    range of them by pointer.  requests: (src, tgt, conn, syn) or (src, tgt,
    conn, syn, alpha) tuples; alpha defaults to `alpha` (else -1)."""

    def __init__(self, requests, alpha: int | None = None):
        n = len(requests)
        nseg = sum(len(r[0]) + len(r[1]) for r in requests)
        self.n = n
        self.segs = (Segment * max(1, nseg))()
        self.S = (NodeSet * max(1, n))()
        self.T = (NodeSet * max(1, n))()
        self.C = (ConnSpec * max(1, n))()
        self.Y = (SynSpec * max(1, n))()
        self.A = (ctypes.c_int32 * max(1, n))()
        base = ctypes.addressof(self.segs)
        k = 0
        try:
            for i, r in enumerate(requests):
                src, tgt, conn, syn = r[:4]
                if conn["rule"] == "assigned_nodes":
                    raise SnncError(-1, "assigned nodes take their pairs through connect_assigned")
                for dst, group in ((self.S, src), (self.T, tgt)):
                    dst[i].seg = ctypes.cast(base + 12 * k, ctypes.POINTER(Segment))
                    dst[i].n_seg = len(group)
                    for h, f, m in group:
                        self.segs[k].host, self.segs[k].first, self.segs[k].n = int(h), int(f), int(m)
                        k += 1
                self.C[i] = ConnSpec(RULES[conn["rule"]], int(conn.get("autapses", True)),
                                     int(conn.get("multapses", True)), 0, int(conn.get("n", 0)),
                                     float(conn.get("p", 0.0)))
                self.Y[i] = SynSpec(_dist(syn.get("weight")), _dist(syn.get("delay")), int(syn.get("port", 0)), 0)
                self.A[i] = int(r[4] if len(r) > 4 else (-1 if alpha is None else alpha))
        except (OverflowError, TypeError, ValueError) as err:
            raise SnncError(-1, f"request argument out of range: {err}") from None

    def __len__(self):
        return self.n

    def at(self, which: str, i: int):
        """Address of element i of array S, T, C, Y or A."""
        arr = getattr(self, which)
        return ctypes.c_void_p(ctypes.addressof(arr) + i * ctypes.sizeof(arr._type_))


class Network:
    """One virtual host's share of a network, built on the current GPU."""

    def __init__(self, P: int, P_local: int, seed: int, dt: float, budget_bytes: int = 0,
                 torch_allocator: bool = True, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the construction library runs on the GPU only")
        self._torch = torch
        self.device = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._alloc = None
        if torch_allocator:
            dev, strm = self.device, self.stream

            def _a(nbytes, _stream, _user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, strm)
                except Exception:   # out of memory: the library reports SNNC_ENOMEM
                    return None

            def _f(ptr, _user):
                torch.cuda.caching_allocator_delete(ptr)

            self._alloc_cbs = (ALLOC_FN(_a), FREE_FN(_f))
            self._alloc = Allocator(self._alloc_cbs[0], self._alloc_cbs[1], None)
        h = ctypes.c_void_p()
        st = lib().snnc_init(ctypes.byref(h), P, P_local, seed & 0xFFFFFFFF, dt,
                             ctypes.byref(self._alloc) if self._alloc is not None else None,
                             ctypes.c_void_p(self.stream.cuda_stream), budget_bytes)
        if st != 0:
            raise SnncError(st, "snnc_init failed")
        self._h = h
        self.P, self.P_local = P, P_local

    def close(self):
        if getattr(self, "_h", None):
            lib().snnc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise SnncError(st, lib().snnc_last_error(self._h).decode())

    def create(self, host: int, n: int) -> tuple:
        seg = Segment()
        self._check(lib().snnc_create(self._h, host, n, ctypes.byref(seg)))
        return (seg.host, seg.first, seg.n)

    def _connect_like(self, name, src, tgt, conn, syn, alpha):
        # one struct.pack per argument group into a buffer reused across calls
        ns, nt = len(src), len(tgt)
        need = _OFF_SEG + 12 * (ns + nt)
        if need > len(getattr(self, "_mb", b"")):
            self._mb = ctypes.create_string_buffer(max(need, 1024))
            self._mb_cid = ctypes.c_uint32.from_buffer(self._mb, _OFF_CID)
        mb = self._mb
        base = ctypes.addressof(mb)
        w = syn.get("weight") or _CONST0
        d = syn.get("delay") or _CONST0
        try:
            _SPEC.pack_into(mb, 0, RULES[conn["rule"]], int(conn.get("autapses", True)),
                            int(conn.get("multapses", True)), 0, int(conn.get("n", 0)), float(conn.get("p", 0.0)),
                            DISTS[w.get("kind", "const")], 0, float(w.get("mean", 0.0)), float(w.get("sd", 0.0)),
                            float(w.get("lo", 0.0)),
                            DISTS[d.get("kind", "const")], 0, float(d.get("mean", 0.0)), float(d.get("sd", 0.0)),
                            float(d.get("lo", 0.0)), int(syn.get("port", 0)), 0)
            seg0 = base + _OFF_SEG
            _NODESETS.pack_into(mb, _OFF_NS, seg0, ns, seg0 + 12 * ns, nt)
            _seg_struct(ns + nt).pack_into(mb, _OFF_SEG, *[int(v) for g in src for v in g],
                                           *[int(v) for g in tgt for v in g])
        except struct.error as err:
            raise SnncError(-1, f"connection argument out of range: {err}") from None
        self._check(lib().packed[name](self._h, base + _OFF_NS, base + _OFF_NS + 16, base, base + _OFF_SYN,
                                       int(alpha), base + _OFF_CID))
        return int(self._mb_cid.value)

    def connect(self, src, tgt, conn, syn, alpha: int = -1) -> int:
        if conn["rule"] == "assigned_nodes":
            return self.connect_assigned(src, tgt, conn["pairs"][0], conn["pairs"][1], syn, alpha)
        return self._connect_like("snnc_connect", src, tgt, conn, syn, alpha)

    def connect_assigned(self, src, tgt, src_pos, tgt_pos, syn, alpha: int = -1) -> int:
        """Assigned nodes: pair i connects position src_pos[i] of src to
        position tgt_pos[i] of tgt (host arrays, copied by the call)."""
        s, s_keep = _nodeset(src)
        t, t_keep = _nodeset(tgt)
        sp = np.ascontiguousarray(src_pos, dtype=np.uint32)
        tp = np.ascontiguousarray(tgt_pos, dtype=np.uint32)
        if sp.shape != tp.shape or sp.ndim != 1:
            raise SnncError(-1, "pair arrays differ in shape")
        ss = SynSpec(_dist(syn.get("weight")), _dist(syn.get("delay")), int(syn.get("port", 0)), 0)
        cid = ctypes.c_uint32()
        self._check(lib().snnc_connect_assigned(self._h, ctypes.byref(s), ctypes.byref(t), sp.ctypes.data,
                                                tp.ctypes.data, int(sp.size), ctypes.byref(ss), int(alpha),
                                                ctypes.byref(cid)))
        return int(cid.value)

    def submit(self, src, tgt, conn, syn, alpha: int = -1) -> int:
        """Served mode: admit and reserve now, generate at the next flush()."""
        return self._connect_like("snnc_submit", src, tgt, conn, syn, alpha)

    def submit_many(self, requests, alpha: int | None = None):
        """Served mode, several requests with one device wait for their counts:
        requests is a list of (src, tgt, conn, syn) or (src, tgt, conn, syn,
        alpha), or a RequestBatch.  Returns one (status, call_id) per request:
        status 0 when admitted, else the request's error code (-3 over
        budget), call_id None when not admitted."""
        batch = requests if isinstance(requests, RequestBatch) else RequestBatch(requests, alpha)
        return self.submit_batch(batch, 0, len(batch))

    def submit_batch(self, batch: "RequestBatch", lo: int, hi: int):
        """snnc_submit_many over requests [lo, hi) of a packed RequestBatch."""
        n = max(0, min(hi, len(batch)) - lo)
        st = (ctypes.c_int32 * max(1, n))()
        ids = (ctypes.c_uint32 * max(1, n))()
        self._check(lib().snnc_submit_many(self._h, n, batch.at("S", lo), batch.at("T", lo), batch.at("C", lo),
                                           batch.at("Y", lo), batch.at("A", lo), st, ids))
        return [(int(st[i]), int(ids[i]) if st[i] == 0 else None) for i in range(n)]

    def connect_packed(self, batch: "RequestBatch", i: int, submit: bool = False) -> int:
        """snnc_connect (or, with submit, snnc_submit) of request i of a packed
        RequestBatch."""
        cid = ctypes.c_uint32()
        self._check(lib().packed["snnc_submit" if submit else "snnc_connect"](self._h, batch.at("S", i).value, batch.at("T", i).value,
                                                 batch.at("C", i).value, batch.at("Y", i).value, int(batch.A[i]),
                                                 ctypes.addressof(cid)))
        return int(cid.value)

    def flush(self):
        self._check(lib().snnc_flush(self._h))

    def poll(self, call_id: int) -> bool:
        done = ctypes.c_int32()
        self._check(lib().snnc_poll(self._h, int(call_id), ctypes.byref(done)))
        return bool(done.value)

    def set_resident_budget(self, nbytes: int):
        self._check(lib().snnc_set_resident_budget(self._h, int(nbytes)))

    def reserve(self, n: int):
        self._check(lib().snnc_reserve(self._h, int(n)))

    def set_memory_level(self, level: int):
        """GPU memory level 0..3 (placement of the maps and image rows, and
        images of used (0) or all passed sources (1..3))."""
        self._check(lib().snnc_set_memory_level(self._h, int(level)))

    def on_host(self, name: str) -> bool:
        which, _ = ARRAYS[name]
        flag = ctypes.c_int32()
        self._check(lib().snnc_array_on_host(self._h, which, ctypes.byref(flag)))
        return bool(flag.value)

    def set_map_policy(self, numbering: int, sources: int, xi: float = 1.0):
        """numbering: 0 canonical, 1 in call order; sources: 0 used, 1
        threshold heuristic with xi, 2 all passed sources."""
        self._check(lib().snnc_set_map_policy(self._h, int(numbering), int(sources), float(xi)))

    def prepare(self):
        self._check(lib().snnc_prepare(self._h))

    def sync(self):
        self._check(lib().snnc_sync(self._h))

    def array_ptr(self, name: str) -> tuple:
        """(pointer, element count) that snnc_get_array hands out for an array."""
        which, _ = ARRAYS[name]
        p, n = ctypes.c_void_p(), ctypes.c_uint64()
        self._check(lib().snnc_get_array(self._h, which, ctypes.byref(p), ctypes.byref(n)))
        return p.value, int(n.value)

    def count(self, name: str) -> int:
        which, _ = ARRAYS[name]
        p, n = ctypes.c_void_p(), ctypes.c_uint64()
        self._check(lib().snnc_get_array(self._h, which, ctypes.byref(p), ctypes.byref(n)))
        return int(n.value)

    def array(self, name: str) -> np.ndarray:
        """Host copy of a result array."""
        which, dt = ARRAYS[name]
        out = np.zeros(self.count(name), dt)
        self._check(lib().snnc_copy_array(self._h, which, out.ctypes.data, out.nbytes))
        return out

    def array_range(self, name: str, first: int, count: int) -> np.ndarray:
        which, dt = ARRAYS[name]
        out = np.zeros(count, dt)
        self._check(lib().snnc_copy_range(self._h, which, int(first), int(count), out.ctypes.data))
        return out

    def tensor(self, name: str):
        """Device copy of a result array as a torch tensor (same dtype widths)."""
        torch = self._torch
        which, dt = ARRAYS[name]
        n = self.count(name)
        tdt = {np.uint32: torch.int32, np.int32: torch.int32, np.uint16: torch.int16, np.float32: torch.float32,
               np.uint64: torch.int64, np.int64: torch.int64}[dt]
        out = torch.empty(n, dtype=tdt, device=f"cuda:{self.device}")
        self._check(lib().snnc_copy_array(self._h, which, ctypes.c_void_p(out.data_ptr()), out.numel() * out.element_size()))
        return out

    def connections_view(self) -> dict:
        """snnc_get_connections: pointers (addresses) and sizes of the sorted
        connections and their first-index array."""
        v = ConnView()
        self._check(lib().snnc_get_connections(self._h, ctypes.byref(v)))
        return {f: getattr(v, f) for f, _ in ConnView._fields_}

    def image_map(self, alpha: int, sigma: int) -> dict:
        """snnc_get_image_map of (alpha, sigma): R, L as host copies (read
        through the returned pointers), img_base and the pointers."""
        R, L = ctypes.c_void_p(), ctypes.c_void_p()
        n, base = ctypes.c_uint64(), ctypes.c_int64()
        self._check(lib().snnc_get_image_map(self._h, int(alpha), int(sigma), ctypes.byref(R), ctypes.byref(n),
                                             ctypes.byref(base), ctypes.byref(L)))
        return {"R_ptr": R.value, "L_ptr": L.value, "n": int(n.value), "img_base": int(base.value),
                "R": self._read(R.value, int(n.value), np.int32, "r_val"),
                "L": self._read(L.value, int(n.value), np.int32, "l_val")}

    def p2p_send(self) -> dict:
        v = P2PView()
        self._check(lib().snnc_get_p2p_send(self._h, ctypes.byref(v)))
        return {f: getattr(v, f) for f, _ in P2PView._fields_}

    def collective(self, alpha: int) -> dict:
        v = CollView()
        self._check(lib().snnc_get_collective(self._h, int(alpha), ctypes.byref(v)))
        return {f: getattr(v, f) for f, _ in CollView._fields_}

    def copy_to_host(self, name: str) -> np.ndarray:
        """snnc_copy_to_host of a whole array into a new numpy array."""
        which, dt = ARRAYS[name]
        out = np.zeros(self.count(name), dt)
        self._check(lib().snnc_copy_to_host(self._h, which, out.ctypes.data if out.size else None, out.nbytes))
        return out

    def _read(self, ptr, n: int, dtype, name: str) -> np.ndarray:
        """Host copy of n elements at a pointer into array `name` that a view
        handed out (through snnc_copy_range at the pointer's offset)."""
        if not n or not ptr:
            return np.zeros(0, dtype)
        base = ctypes.c_void_p()
        cnt = ctypes.c_uint64()
        self._check(lib().snnc_get_array(self._h, ARRAYS[name][0], ctypes.byref(base), ctypes.byref(cnt)))
        first = (ptr - base.value) // np.dtype(dtype).itemsize
        return self.array_range(name, int(first), n)

    def stats(self) -> dict:
        s = Stats()
        self._check(lib().snnc_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def set_timing(self, on):
        """False/True (0/1): off / every launch; 2: the radix-sort passes only."""
        self._check(lib().snnc_set_timing(self._h, int(on)))

    def kernel_times(self) -> dict:
        cap = 64
        names = (ctypes.c_char * 48 * cap)()
        launches = (ctypes.c_uint64 * cap)()
        ms = (ctypes.c_double * cap)()
        n = ctypes.c_uint32()
        self._check(lib().snnc_kernel_times(self._h, cap, names, launches, ms, ctypes.byref(n)))
        return {names[i].value.decode(): (int(launches[i]), float(ms[i])) for i in range(min(n.value, cap))}

    def tune(self, key: str, value: int):
        self._check(lib().snnc_tune(self._h, key.encode(), int(value)))

    @staticmethod
    def _dptr(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    def spike_packets(self, kind: int, spikes, mult=None) -> dict:
        """Packets of one time step from device tensors spikes / mult (int32
        holding unsigned ids and counts): kind 0 per target host (T/P), kind 1
        per group (G/Q).  Returns tensors off, pos, mult."""
        torch = self._torch
        dev = spikes.device
        n_dest = self.P if kind == 0 else int(self.count("groups"))
        off = torch.empty(n_dest + 1, dtype=torch.int64, device=dev)
        cap = max(1, int(self.count("t_val" if kind == 0 else "q_val")))
        for _ in range(2):
            pos = torch.empty(cap, dtype=torch.int32, device=dev)
            mo = torch.empty(cap, dtype=torch.int32, device=dev)
            n_out = ctypes.c_uint64()
            st = lib().snnc_spike_packets(self._h, kind, self._dptr(spikes), self._dptr(mult), spikes.numel(),
                                          self._dptr(off), self._dptr(pos), self._dptr(mo), cap, ctypes.byref(n_out))
            if st != 0 and n_out.value > cap:
                cap = n_out.value
                continue
            self._check(st)
            return {"off": off, "pos": pos[:n_out.value], "mult": mo[:n_out.value]}
        raise SnncError(-1, "packet capacity")

    def deliver(self, kind: int, host, pos, mult=None, grp=None, events: bool = True) -> dict:
        """Delivery of received entries (device int32 tensors): image and row
        per entry, and the (target, delay, weight x multiplicity) events."""
        torch = self._torch
        dev = host.device
        n = host.numel()
        image = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        rb = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
        re = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
        cap = max(1, n * 64)
        for _ in range(2):
            et = torch.empty(cap, dtype=torch.int32, device=dev) if events else None
            ed = torch.empty(cap, dtype=torch.int16, device=dev) if events else None
            ew = torch.empty(cap, dtype=torch.float32, device=dev) if events else None
            n_ev = ctypes.c_uint64()
            st = lib().snnc_deliver(self._h, kind, self._dptr(grp), self._dptr(host), self._dptr(pos),
                                    self._dptr(mult), n, self._dptr(image), self._dptr(rb), self._dptr(re),
                                    self._dptr(et), self._dptr(ed), self._dptr(ew), cap if events else 0,
                                    ctypes.byref(n_ev))
            if st != 0 and events and n_ev.value > cap:
                cap = n_ev.value
                continue
            self._check(st)
            out = {"image": image[:n], "row_begin": rb[:n], "row_end": re[:n], "n_events": n_ev.value}
            if events:
                out.update(tgt=et[:n_ev.value], delay=ed[:n_ev.value], weight=ew[:n_ev.value])
            return out
        raise SnncError(-1, "event capacity")

    def autotune_sort(self, n: int, bits: int) -> dict:
        """Pick the fastest radix-pass algorithm and tile shape for n keys of
        `bits` sorted bits (cached per size class for the process)."""
        m, v, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        self._check(lib().snnc_autotune_sort(self._h, int(n), int(bits), ctypes.byref(m), ctypes.byref(v),
                                             ctypes.byref(ms)))
        return {"sort_mode": m.value, "sort_variant": v.value, "ms": ms.value}

    def autotune_fused(self, n: int) -> dict:
        """Pick the grid of the persistent batch launch (workgroups per
        compute unit) on a synthetic batch of about n connections (cached
        per device for the process)."""
        w, ms = ctypes.c_int32(), ctypes.c_float()
        self._check(lib().snnc_autotune_fused(self._h, int(n), ctypes.byref(w), ctypes.byref(ms)))
        return {"fused_wgs_per_cu": w.value, "ms": ms.value}

    def sort_pairs(self, keys, vals, bit_lo: int, bit_hi: int):
        """Stable radix sort of device tensors keys (int64) / vals (int32) by
        key bits [bit_lo, bit_hi); returns the sorted (keys, vals) tensors."""
        torch = self._torch
        kt, vt = torch.empty_like(keys), torch.empty_like(vals)
        where = ctypes.c_int32()
        self._check(lib().snnc_sort_pairs(self._h, ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
                                          ctypes.c_void_p(kt.data_ptr()), ctypes.c_void_p(vt.data_ptr()),
                                          keys.numel(), bit_lo, bit_hi, ctypes.byref(where)))
        return (kt, vt) if where.value else (keys, vals)

    def sort_pairs_noalloc(self, keys, vals, keys_tmp, vals_tmp, bit_lo: int, bit_hi: int):
        """snnc_sort_pairs_noalloc on caller tensors (keys int64, vals int32,
        and ping-pong buffers of the same sizes); the library allocates
        nothing.  Returns the (keys, vals) pair that holds the result."""
        where = ctypes.c_int32()
        self._check(lib().snnc_sort_pairs_noalloc(
            self._h, ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
            ctypes.c_void_p(keys_tmp.data_ptr()), ctypes.c_void_p(vals_tmp.data_ptr()), keys.numel(), bit_lo, bit_hi,
            ctypes.byref(where)))
        return (keys_tmp, vals_tmp) if where.value else (keys, vals)

    def philox_blocks(self, seed: int, call_id: int, e_begin: int, purpose: int, n: int) -> np.ndarray:
        torch = self._torch
        out = torch.empty(4 * n, dtype=torch.int32, device=f"cuda:{self.device}")
        self._check(lib().snnc_philox_blocks(self._h, seed, call_id, e_begin, purpose, n,
                                             ctypes.c_void_p(out.data_ptr())))
        return out.cpu().numpy().view(np.uint32).reshape(n, 4)


def run_script(script: dict, P_local: int, prepare: bool = True, skip_invalid: bool = False, **kw) -> Network:
    """Replay a workload script on the GPU for host P_local."""
    net = Network(script["P"], P_local, script["seed"], script["dt"], **kw)
    if script.get("memory_level") is not None:
        net.set_memory_level(script["memory_level"])
    if script.get("map_policy") is not None:
        net.set_map_policy(*script["map_policy"])
    for key, value in script.get("tune", {}).items():
        net.tune(key, value)
    net.rejected = []
    for k, op in enumerate(script["ops"]):
        if op[0] == "create":
            net.create(op[1], op[2])
            continue
        _, src, tgt, conn, syn, alpha = op
        try:
            net.connect(src, tgt, conn, syn, alpha)
        except SnncError as err:
            if not skip_invalid or err.code not in (-1, -5):
                raise
            net.rejected.append((k, err.code))
    if prepare:
        net.prepare()
    return net
