"""Host logic of the Python binding: connect/submit pack their arguments into
one reused buffer in the C layout of snnc_nodeset / snnc_conn_spec /
snnc_syn_spec.  A stand-in for the library reads the buffer back through the
ctypes structs (the declared layout) and must see the same values as the
per-struct marshalling would give; out-of-range values raise SnncError."""
import ctypes

import pytest

import paper_2512_09502_amd as snnc
from paper_2512_09502_amd import workloads as W


class _Reader:
    def __init__(self):
        self.seen = None

    def __call__(self, h, ps, pt, pc, pss, alpha, pcid):
        S, T = snnc.NodeSet.from_address(ps), snnc.NodeSet.from_address(pt)
        c, y = snnc.ConnSpec.from_address(pc), snnc.SynSpec.from_address(pss)
        self.seen = ([(S.seg[i].host, S.seg[i].first, S.seg[i].n) for i in range(S.n_seg)],
                     [(T.seg[i].host, T.seg[i].first, T.seg[i].n) for i in range(T.n_seg)],
                     (c.kind, c.allow_autapses, c.allow_multapses, c.reserved, c.n, c.p),
                     tuple((d.kind, d.reserved, d.mean, d.sd, d.lo) for d in (y.weight, y.delay_ms)) +
                     (y.port, y.reserved), alpha)
        ctypes.c_uint32.from_address(pcid).value = 4242
        return 0


class _FakeLib:
    def __init__(self, reader):
        self.packed = {"snnc_connect": reader, "snnc_submit": reader}


class _Net(snnc.Network):
    def __init__(self):   # no device: only the marshalling is exercised
        self._h = None

    def _check(self, st):
        assert st == 0


@pytest.fixture
def net(monkeypatch):
    reader = _Reader()
    monkeypatch.setattr(snnc, "_lib", _FakeLib(reader))
    n = _Net()
    n.reader = reader
    return n


def _expected(src, tgt, conn, syn, alpha):
    d = [snnc._dist(syn.get("weight")), snnc._dist(syn.get("delay"))]
    return ([tuple(map(int, g)) for g in src], [tuple(map(int, g)) for g in tgt],
            (snnc.RULES[conn["rule"]], int(conn.get("autapses", True)), int(conn.get("multapses", True)), 0,
             int(conn.get("n", 0)), float(conn.get("p", 0.0))),
            tuple((x.kind, 0, x.mean, x.sd, x.lo) for x in d) + (int(syn.get("port", 0)), 0), alpha)


def test_layout_matches_the_structs():
    assert ctypes.sizeof(snnc.ConnSpec) == 32 and ctypes.sizeof(snnc.SynSpec) == 72
    assert ctypes.sizeof(snnc.NodeSet) == 16 and ctypes.sizeof(snnc.Segment) == 12


@pytest.mark.parametrize("name", ["multiarea_p2p", "balanced_small", "served_requests"] +
                         [f"random_tiny:{s}" for s in range(12)])
def test_packed_arguments_read_back(net, name):
    base, _, arg = name.partition(":")
    script = getattr(W, base)(*([int(arg)] if arg else []))
    n = 0
    for op in script["ops"]:
        if op[0] != "connect" or op[3]["rule"] == "assigned_nodes":
            continue
        _, src, tgt, conn, syn, alpha = op
        for entry in ("snnc_connect", "snnc_submit"):
            assert net._connect_like(entry, src, tgt, conn, syn, alpha) == 4242
            assert net.reader.seen == _expected(src, tgt, conn, syn, alpha)
        n += 1
        if n > 400:
            break
    assert n > 0


def test_buffer_grows_with_segments(net):
    src = [(h, 0, 5) for h in range(300)]
    conn, syn = {"rule": "fixed_indegree", "n": 3}, {}
    assert net._connect_like("snnc_connect", src, [(0, 0, 5)], conn, syn, 2) == 4242
    assert net.reader.seen == _expected(src, [(0, 0, 5)], conn, syn, 2)
    assert net._connect_like("snnc_connect", [], [], {"rule": "one_to_one"}, syn, -1) == 4242
    assert net.reader.seen[:2] == ([], [])


@pytest.mark.parametrize("bad", [[(0, -1, 3)], [(2**32, 0, 3)], [(0, 0, 3, 4)]])
def test_out_of_range_values_raise(net, bad):
    with pytest.raises(snnc.SnncError) as e:
        net._connect_like("snnc_connect", bad, [(0, 0, 3)], {"rule": "one_to_one"}, {}, -1)
    assert e.value.code == -1
