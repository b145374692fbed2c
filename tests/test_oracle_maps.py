"""Pins of the oracle's distributed structures: the union of all hosts' shares
equals a one-host build of the same network, the image map is a bijection onto
the used remote sources, the point-to-point sequences on the source host equal
the maps on the target host (map alignment), the collective H/I/G/Q arrays
satisfy their definitions, and the paper's worked examples (Figs. 1, 2 and the
App. E tables) come out as printed."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2512_09502_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _flatten_to_one_host(script, drop_ops=()):
    """Same network on a single host: every neuron keeps its creation order."""
    creates = []
    for op in script["ops"]:
        if op[0] == "create":
            creates.append(op)
    # new first of each (host, orig_first)
    new_first = {}
    cursor = 0
    per_host_cursor = {}
    for _, h, n in creates:
        f = per_host_cursor.get(h, 0)
        new_first[(h, f)] = (cursor, n)
        per_host_cursor[h] = f + n
        cursor += n

    def remap_seg(h, f, n):
        out = []
        while n > 0:
            for (hh, ff), (nf, nn) in new_first.items():
                if hh == h and ff <= f < ff + nn:
                    k = min(n, ff + nn - f)
                    out.append((0, nf + (f - ff), k))
                    f += k
                    n -= k
                    break
            else:
                raise AssertionError("segment outside creates")
        return out

    ops = []
    for k, op in enumerate(script["ops"]):
        if op[0] == "create":
            ops.append(("create", 0, op[2]))
        elif k not in drop_ops:
            _, src, tgt, conn, syn, alpha = op
            s2 = [x for s in src for x in remap_seg(*s)]
            t2 = [x for t in tgt for x in remap_seg(*t)]
            ops.append(("connect", s2, t2, conn, syn, alpha))
    out = dict(script)
    out["P"] = 1
    out["ops"] = ops
    return out, remap_seg


def _records(net, script_host_of_local):
    """(call, e) keyed generation records with the target as a global id"""
    off = net.array("call_off").astype(np.int64)
    call = np.repeat(np.arange(off.size - 1), np.diff(off))
    return {
        "call": call, "e": net.array("gen_e").astype(np.int64),
        "src": net.array("gen_src").astype(np.int64),
        "tgt": np.array([script_host_of_local(int(t)) for t in net.array("gen_tgt")], np.int64),
        "delay": net.array("gen_delay"), "weight": net.array("gen_weight"),
    }


def _sorted_concat(recs):
    cat = {k: np.concatenate([r[k] for r in recs]) for k in recs[0]}
    order = np.lexsort((cat["e"], cat["call"]))
    return {k: v[order] for k, v in cat.items()}


@pytest.mark.parametrize("seed", range(12))
def test_union_of_shares_equals_one_host_build(seed):
    script = W.random_tiny(seed, P=int(2 + seed % 3))
    P = script["P"]
    shares = [oracle.run_script(script, pl, skip_invalid=True) for pl in range(P)]
    rejected = {k for k, _ in shares[0].rejected}
    for sh in shares[1:]:
        assert {k for k, _ in sh.rejected} == rejected     # validation is host-independent
    flat, remap_seg = _flatten_to_one_host(script, drop_ops=rejected)
    one = oracle.run_script(flat, 0)
    recs = [_records(sh, lambda t, pl=pl: remap_seg(pl, t, 1)[0][1]) for pl, sh in enumerate(shares)]
    a = _sorted_concat(recs)
    b = _sorted_concat([_records(one, lambda t: t)])
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def _set_lookup(segs, ordinal):
    for h, f, n in segs:
        if ordinal < n:
            return h, f + ordinal
        ordinal -= n
    raise AssertionError


def _decode(net, src_prime, M_local, P):
    """image index -> (a, sigma, source local id) through img_base / R"""
    r_off = net.array("r_off").astype(np.int64)
    r_val = net.array("r_val")
    img_base = net.array("img_base")
    k = int(np.searchsorted(img_base + np.diff(r_off), src_prime, side="right"))
    a, sigma = divmod(k, P)
    return a, sigma, int(r_val[r_off[k] + (src_prime - img_base[k])])


@pytest.mark.parametrize("seed", range(8))
def test_image_map_bijection_and_remap(seed):
    script = W.random_tiny(100 + seed, P=3)
    P = script["P"]
    for pl in range(P):
        net = oracle.run_script(script, pl, skip_invalid=True)
        M_local = net.neurons(pl)
        r_off = net.array("r_off").astype(np.int64)
        r_val = net.array("r_val")
        img_base = net.array("img_base")
        # R strictly increasing per (a, sigma); images numbered after the local neurons
        for k in range(r_off.size - 1):
            seg = r_val[r_off[k]:r_off[k + 1]]
            assert (np.diff(seg) > 0).all()
            assert img_base[k] == M_local + r_off[k]
            if k % P == pl:
                assert seg.size == 0
        # expected multiset of (a, sigma, s, tgt, delay, weight) from the generation records
        rejected = {k for k, _ in net.rejected}
        ops = [op for k, op in enumerate(script["ops"]) if op[0] == "connect" and k not in rejected]
        off = net.array("call_off").astype(np.int64)
        gs, gt = net.array("gen_src"), net.array("gen_tgt")
        gd, gw = net.array("gen_delay"), net.array("gen_weight")
        expect, used = [], set()
        for c, op in enumerate(ops):
            for i in range(off[c], off[c + 1]):
                h, l = _set_lookup(op[1], int(gs[i]))
                a = op[5] + 1
                key = (a, h, l) if h != pl else (-1, h, l)
                if h != pl:
                    used.add((a, h, l))
                expect.append(key + (int(gt[i]), int(gd[i]), float(gw[i])))
        assert r_val.size == len(used)                        # one image per used remote source
        src = net.array("src")
        tgt, dl, wt = net.array("tgt"), net.array("delay"), net.array("weight")
        got = []
        for i in range(src.size):
            s = int(src[i])
            key = (-1, pl, s) if s < M_local else _decode(net, s, M_local, P)
            got.append(key + (int(tgt[i]), int(dl[i]), float(wt[i])))
        assert sorted(got) == sorted(expect)
        # source-major, then target; first-index array consistent with counts
        pairs = src.astype(np.int64) * 2**32 + tgt.astype(np.int64)
        assert (np.diff(pairs) >= 0).all()
        rp = net.array("row_ptr").astype(np.int64)
        assert rp[0] == 0 and rp[-1] == src.size
        assert (np.diff(rp) == np.bincount(src, minlength=rp.size - 1)).all()


@pytest.mark.parametrize("seed", range(6))
def test_p2p_map_alignment_across_hosts(seed):
    """S_{tau,sigma} stored on sigma equals R_{tau,sigma} stored on tau."""
    script = W.multiarea_p2p(P=4, n_e=40, n_i=10, k_e=8, k_i=2, k_remote_max=6, seed=50 + seed)
    P = script["P"]
    nets = [oracle.run_script(script, pl) for pl in range(P)]
    for sigma in range(P):
        s_off = nets[sigma].array("s_off").astype(np.int64)
        s_val = nets[sigma].array("s_val")
        for tau in range(P):
            S = s_val[s_off[tau]:s_off[tau + 1]]
            r_off = nets[tau].array("r_off").astype(np.int64)
            R = nets[tau].array("r_val")[r_off[sigma]:r_off[sigma + 1]]   # a = 0 block
            np.testing.assert_array_equal(S, R, err_msg=f"sigma={sigma} tau={tau}")
        # T/P: every (tau, i) pair of neuron s points at S_tau[i] == s, tau ascending
        tp = nets[sigma].array("tp_ptr").astype(np.int64)
        T, Pp = nets[sigma].array("t_val"), nets[sigma].array("p_val")
        assert tp[-1] == s_off[-1]
        for s in range(tp.size - 1):
            taus = T[tp[s]:tp[s + 1]]
            assert (np.diff(taus.astype(np.int64)) > 0).all()
            for tau, i in zip(taus, Pp[tp[s]:tp[s + 1]]):
                assert s_val[s_off[tau] + i] == s


def test_collective_arrays_definitions():
    script = W.balanced_collective(P=5, n_e=40, n_i=10, k_e=9, k_i=3)
    P = script["P"]
    nets = [oracle.run_script(script, pl) for pl in range(P)]
    H0 = nets[0].array("h_val")
    for net in nets[1:]:
        np.testing.assert_array_equal(net.array("h_val"), H0)          # H mirrored on all members
        np.testing.assert_array_equal(net.array("h_off"), nets[0].array("h_off"))
    for pl, net in enumerate(nets):
        assert net.array("groups").tolist() == [0]
        h_off = net.array("h_off").astype(np.int64)
        H, I = net.array("h_val"), net.array("i_val")
        r_off = net.array("r_off").astype(np.int64)
        R, base = net.array("r_val"), net.array("img_base")
        for sigma in range(P):
            h = H[h_off[sigma]:h_off[sigma + 1]]
            i = I[h_off[sigma]:h_off[sigma + 1]]
            assert (h == np.arange(50)).all()           # the union of the passed sources, sorted
            k = P + sigma                               # a = alpha + 1 = 1
            r = R[r_off[k]:r_off[k + 1]]
            if sigma == pl:
                assert (i == -1).all()
                continue
            has = np.isin(h, r)
            assert ((i >= 0) == has).all()              # -1 exactly where there is no image
            assert (i[has] == base[k] + np.searchsorted(r, h[has])).all()
        gq = net.array("gq_ptr").astype(np.int64)
        assert (np.diff(gq) == 1).all()                 # every local neuron reports to group 0
        assert (net.array("g_val") == 0).all()
        assert (net.array("q_val") == np.arange(50)).all()


def test_app_e_send_tables():
    g = json.load(open(os.path.join(GOLDEN, "app_e_send_tables.json")))
    P, M = g["P"], 800
    lists = []
    for tau in range(P):
        pos = {int(s): p for s, p in g["positions"].get(str(tau), {}).items()}
        n = (max(pos.values()) + 1) if pos else 0
        # fill the other positions with ascending ids that keep the given ones in place
        free = [x for x in range(M) if x not in pos]
        lst, fi = [], 0
        for i in range(n):
            want = [s for s, p in pos.items() if p == i]
            if want:
                lst.append(want[0])
            else:
                lo = lst[-1] + 1 if lst else 0
                nxt = min([s for s, p in pos.items() if p > i], default=M)
                cand = [x for x in free if lo <= x < nxt]
                lst.append(cand[0])
                free.remove(cand[0])
        assert lst == sorted(lst)
        lists.append(lst)
    ptr, which, where = oracle.transpose_lists(lists, M)
    for s, exp in g["expect"].items():
        s = int(s)
        a, b = int(ptr[s]), int(ptr[s + 1])
        assert which[a:b].tolist() == exp["T"]
        assert where[a:b].tolist() == exp["P"]


def test_app_e_delivery_blocks():
    g = json.load(open(os.path.join(GOLDEN, "app_e_delivery_blocks.json")))
    c = np.array(g["connections"])
    out = oracle.sort_csr(c[:, 0], c[:, 1], c[:, 2], np.ones(len(c)), 1000)
    rp = out["row_ptr"].astype(np.int64)
    for s, exp in g["expect"].items():
        s = int(s)
        assert out["tgt"][rp[s]:rp[s + 1]].tolist() == exp["targets"]
        assert out["delay"][rp[s]:rp[s + 1]].tolist() == exp["delays"]


SYN = {"weight": {"kind": "const", "mean": 1.0}, "delay": {"kind": "const", "mean": 0.1}}


def test_fig1_point_to_point_example():
    """Fig. 1: neuron 0 of rank 2 has images on ranks 0 and 1 at map position
    0 in both, and neuron 1 of rank 0 is image neuron 2 on rank 1 (here rank 1
    holds two neurons, so its first image index is 2)."""
    sizes = {0: 3, 1: 2, 2: 3}
    script = {"P": 3, "seed": 1, "dt": 0.1, "ops": [("create", h, n) for h, n in sizes.items()] + [
        ("connect", [(2, 0, 1)], [(0, 0, 1)], {"rule": "one_to_one"}, SYN, -1),
        ("connect", [(2, 0, 1)], [(1, 0, 1)], {"rule": "one_to_one"}, SYN, -1),
        ("connect", [(0, 1, 1)], [(1, 1, 1)], {"rule": "one_to_one"}, SYN, -1)]}
    nets = [oracle.run_script(script, pl) for pl in range(3)]
    P = 3
    r0 = nets[0].array("r_off").astype(np.int64)
    assert nets[0].array("r_val")[r0[2]:r0[3]].tolist() == [0]          # R_{0,2} = (0)
    r1 = nets[1].array("r_off").astype(np.int64)
    assert nets[1].array("r_val")[r1[2]:r1[3]].tolist() == [0]          # R_{1,2} = (0)
    assert nets[1].array("r_val")[r1[0]:r1[1]].tolist() == [1]          # R_{1,0} = (1)
    assert int(nets[1].array("img_base")[0]) == 2                        # L_{1,0} = (2)
    src = nets[1].array("src")
    assert 2 in src.tolist()
    # T/P of neuron 0 on rank 2: targets (0, 1), positions (0, 0)
    tp = nets[2].array("tp_ptr").astype(np.int64)
    assert nets[2].array("t_val")[tp[0]:tp[1]].tolist() == [0, 1]
    assert nets[2].array("p_val")[tp[0]:tp[1]].tolist() == [0, 0]
    assert P == 3


def test_fig2_collective_example():
    """Fig. 2: neuron 0 of rank 2 reports to group 0 at position Q = 0 of H_{0,2}."""
    script = {"P": 3, "seed": 1, "dt": 0.1, "ops": [("create", h, 3) for h in range(3)] + [
        ("connect", [(2, 0, 3)], [(0, 0, 3), (1, 0, 3)], {"rule": "fixed_indegree", "n": 2}, SYN, 0)]}
    net = oracle.run_script(script, 2)
    gq = net.array("gq_ptr").astype(np.int64)
    assert net.array("g_val")[gq[0]:gq[1]].tolist() == [0]
    assert net.array("q_val")[gq[0]:gq[1]].tolist() == [0]
    h_off = net.array("h_off").astype(np.int64)
    assert net.array("h_val")[h_off[2]:h_off[3]].tolist() == [0, 1, 2]
