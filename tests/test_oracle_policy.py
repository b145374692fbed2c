"""Pins of the oracle's map policies (Methods, point-to-point creation
subsection): which remote sources get an image (only the flagged, i.e. used,
ones; all passed ones; or the threshold heuristic deciding per call), and
how images are numbered (canonical, or the paper's incremental numbering in
call order).

The expected maps are computed here by brute force from the generation
records with a first-use formulation (each image source's first call, then
the order), not by replaying the oracle's append-and-resort steps; the
threshold heuristic is pinned on hand-made calls whose outcome is fixed by
the ratio alone."""
import numpy as np
import pytest

import oracle
from paper_2512_09502_amd import workloads as W

CONST = {"weight": {"kind": "const", "mean": 1.0}, "delay": {"kind": "const", "mean": 1.0}}


def _with_policy(script, pol):
    s = dict(script)
    s["map_policy"] = pol
    return s


def _set_lookup(segs, ordinal):
    for h, f, n in segs:
        if ordinal < n:
            return h, f + ordinal
        ordinal -= n
    raise AssertionError


def _calls(script, net):
    rejected = {k for k, _ in net.rejected}
    return [op for k, op in enumerate(script["ops"]) if op[0] == "connect" and k not in rejected]


def _expected_images(script, net, pl, sources, numbering):
    """{(a, sigma, s): L} by first use: a source's image comes from the first
    call (in call order) with targets on pl that flags it (used sources, with
    sources == 0) or passes it (sources == 2); images are ordered by
    (first call, sigma, s) or canonically by (a, sigma, s)."""
    P = script["P"]
    M_local = net.neurons(pl)
    off = net.array("call_off").astype(np.int64)
    gs = net.array("gen_src")
    first = {}
    for c, op in enumerate(_calls(script, net)):
        _, src, tgt, conn, syn, alpha = op
        if sum(n for h, f, n in tgt if h == pl) == 0:
            continue
        a = alpha + 1
        if sources == 0:
            cand = {_set_lookup(src, int(gs[i])) for i in range(off[c], off[c + 1])}
        else:
            cand = {(h, f + x) for h, f, n in src for x in range(n)}
        for h, s in cand:
            if h != pl and (a, h, s) not in first:
                first[(a, h, s)] = c
    if numbering == 1:
        order = sorted(first, key=lambda k: (first[k], k[1], k[2]))
    else:
        order = sorted(first)
    assert len(order) == len(set(order))
    return {k: M_local + i for i, k in enumerate(order)}, P, M_local


def _maps(net, P):
    r_off = net.array("r_off").astype(np.int64)
    R, L = net.array("r_val"), net.array("l_val")
    out = {}
    for k in range(r_off.size - 1):
        a, sigma = divmod(k, P)
        r = R[r_off[k]:r_off[k + 1]]
        assert (np.diff(r) > 0).all()                    # each map sorted by R
        for i in range(r.size):
            out[(a, sigma, int(r[i]))] = int(L[r_off[k] + i])
    return out


@pytest.mark.parametrize("numbering", [0, 1])
@pytest.mark.parametrize("sources", [0, 2])
@pytest.mark.parametrize("seed", range(6))
def test_maps_match_first_use_brute_force(seed, sources, numbering):
    script = _with_policy(W.random_tiny(300 + seed, P=3), (numbering, sources, 1.0))
    for pl in range(3):
        net = oracle.run_script(script, pl, skip_invalid=True)
        expect, P, M_local = _expected_images(script, net, pl, sources, numbering)
        assert _maps(net, P) == expect
        base = net.array("img_base")
        if numbering == 1:
            assert (base == -1).all()
        else:
            r_off = net.array("r_off").astype(np.int64)
            assert (base == M_local + r_off[:-1]).all()


@pytest.mark.parametrize("pol", [(0, 0, 1.0), (1, 0, 1.0), (0, 1, 1.0), (1, 1, 1.0), (0, 2, 1.0), (1, 2, 1.0)])
@pytest.mark.parametrize("seed", range(4))
def test_remap_decodes_under_every_policy(seed, pol):
    """Every sorted connection's source' leads back through (R, L) to the
    source it was drawn with; L is a bijection onto [M_local, M_local + n_img)."""
    script = _with_policy(W.random_tiny(400 + seed, P=3), pol)
    for pl in range(3):
        net = oracle.run_script(script, pl, skip_invalid=True)
        P, M_local = 3, net.neurons(pl)
        maps = _maps(net, P)
        inv = {v: k for k, v in maps.items()}
        assert sorted(inv) == list(range(M_local, M_local + len(maps)))
        off = net.array("call_off").astype(np.int64)
        gs, gt = net.array("gen_src"), net.array("gen_tgt")
        gd, gw = net.array("gen_delay"), net.array("gen_weight")
        expect = []
        for c, op in enumerate(_calls(script, net)):
            for i in range(off[c], off[c + 1]):
                h, s = _set_lookup(op[1], int(gs[i]))
                key = (-1, h, s) if h == pl else (op[5] + 1, h, s)
                expect.append(key + (int(gt[i]), int(gd[i]), float(gw[i])))
        src, tgt = net.array("src"), net.array("tgt")
        dl, wt = net.array("delay"), net.array("weight")
        got = [((-1, pl, int(s)) if s < M_local else inv[int(s)]) + (int(t), int(d), float(w))
               for s, t, d, w in zip(src, tgt, dl, wt)]
        assert sorted(got) == sorted(expect)
        pairs = src.astype(np.int64) * 2**32 + tgt.astype(np.int64)
        assert (np.diff(pairs) >= 0).all()
        rp = net.array("row_ptr").astype(np.int64)
        assert rp.size == M_local + len(maps) + 1 and rp[-1] == src.size
        assert (np.diff(rp) == np.bincount(src, minlength=rp.size - 1)).all()


def test_single_call_numbering_is_the_canonical_one():
    """With one remote call, numbering in call order (sigma, then s) is the
    canonical (a, sigma, s) order."""
    b = W._Builder(4, seed=77)
    pops = [b.create(h, 30) for h in range(4)]
    b.connect(pops, pops, {"rule": "fixed_indegree", "n": 7}, CONST, -1)
    script = b.script("one_call")
    for pl in range(4):
        nets = [oracle.run_script(_with_policy(script, (num, src, 1.0)), pl) for num in (0, 1) for src in (0, 2)]
        for name in ("r_off", "r_val", "l_val", "src", "tgt", "row_ptr", "s_off", "s_val", "t_val", "p_val"):
            np.testing.assert_array_equal(nets[0].array(name), nets[2].array(name), err_msg=name)   # used
            np.testing.assert_array_equal(nets[1].array(name), nets[3].array(name), err_msg=name)   # all passed


def test_incremental_numbering_follows_call_order():
    """Two calls: the images of the second call's new sources come after all
    images of the first call, even when their ids are smaller."""
    b = W._Builder(2, seed=5)
    hi_src = b.create(0, 20)          # ids 0..19 on host 0
    tgt = b.create(1, 10)
    b.connect([(0, 10, 10)], [tgt], {"rule": "one_to_one"}, CONST, -1)     # sources 10..19 first
    b.connect([(0, 0, 10)], [tgt], {"rule": "one_to_one"}, CONST, -1)      # then 0..9
    script = b.script("two_calls")
    inc = oracle.run_script(_with_policy(script, (1, 0, 1.0)), 1)
    can = oracle.run_script(_with_policy(script, (0, 0, 1.0)), 1)
    np.testing.assert_array_equal(inc.array("r_val"), np.arange(20))
    np.testing.assert_array_equal(can.array("r_val"), np.arange(20))
    np.testing.assert_array_equal(can.array("l_val"), 10 + np.arange(20))
    np.testing.assert_array_equal(inc.array("l_val"), 10 + np.r_[np.arange(10, 20), np.arange(10)])
    assert hi_src == (0, 0, 20)


def _threshold_case(conn, tgt_segments, xi, pl=1):
    """100 sources on host 0; the call's targets as given; returns the map of
    host 0 on host pl under the threshold heuristic and under both fixed
    policies, and S_{pl,0} on host 0."""
    b = W._Builder(2, seed=11)
    b.create(0, 100)
    b.create(1, 10)
    b.connect([(0, 0, 100)], tgt_segments, conn, CONST, -1)
    script = b.script("xi")
    out = {}
    for name, pol in (("xi", (0, 1, xi)), ("used", (0, 0, xi)), ("all", (0, 2, xi))):
        net = oracle.run_script(_with_policy(script, pol), pl)
        r_off = net.array("r_off").astype(np.int64)
        out[name] = net.array("r_val")[r_off[0]:r_off[1]]
        src_net = oracle.run_script(_with_policy(script, pol), 0)
        s_off = src_net.array("s_off").astype(np.int64)
        np.testing.assert_array_equal(src_net.array("s_val")[s_off[pl]:s_off[pl + 1]], out[name])
    return out


# (connection rule, targets, flagged?) -- ratio = estimated connections on host 1 / 100 sources
THRESHOLD_CASES = [
    ({"rule": "fixed_indegree", "n": 2}, [(1, 0, 10)], True),              # 2 * 10 / 100 = 0.2
    ({"rule": "fixed_indegree", "n": 20}, [(1, 0, 10)], False),            # 20 * 10 / 100 = 2
    ({"rule": "fixed_indegree", "n": 9}, [(1, 0, 10)], True),              # 0.9
    ({"rule": "fixed_indegree", "n": 10}, [(1, 0, 10)], False),            # exactly 1: not below
    ({"rule": "pairwise_bernoulli", "p": 0.05}, [(1, 0, 10)], True),       # p N_t = 0.5
    ({"rule": "pairwise_bernoulli", "p": 0.2}, [(1, 0, 10)], False),       # 2
    ({"rule": "fixed_total_number", "n": 50}, [(1, 0, 10)], True),         # 0.5
    ({"rule": "fixed_total_number", "n": 150}, [(1, 0, 10)], False),       # 1.5
    ({"rule": "fixed_outdegree", "n": 1}, [(1, 0, 10), (0, 0, 90)], False),   # uses all sources
    ({"rule": "one_to_one"}, [(1, 0, 10), (0, 0, 90)], False),                # uses all sources
    # assigned nodes: the pairs with a target on host 1, per source
    ({"rule": "assigned_nodes", "pairs": (list(range(50)), [i % 10 for i in range(50)])}, [(1, 0, 10)], True),
    ({"rule": "assigned_nodes", "pairs": ([i % 90 for i in range(150)], [i % 10 for i in range(150)])},
     [(1, 0, 10)], False),                                                      # 1.5
    ({"rule": "assigned_nodes", "pairs": ([i % 60 for i in range(230)], [i % 10 if i < 30 else 10 + i % 90
                                                                          for i in range(230)])},
     [(1, 0, 10), (0, 0, 90)], True),                                           # 30 of 230 on host 1: 0.3
]


@pytest.mark.parametrize("conn,tgt,flagged", THRESHOLD_CASES)
def test_threshold_heuristic(conn, tgt, flagged):
    out = _threshold_case(conn, tgt, 1.0)
    np.testing.assert_array_equal(out["all"], np.arange(100))
    assert out["used"].size < 100                  # every case leaves some source unused on host 1
    np.testing.assert_array_equal(out["xi"], out["used"] if flagged else out["all"])


def test_threshold_extremes():
    conn, tgt = {"rule": "fixed_indegree", "n": 2}, [(1, 0, 10)]
    assert _threshold_case(conn, tgt, 0.0)["xi"].size == 100            # nothing is below 0
    big = _threshold_case({"rule": "fixed_indegree", "n": 20}, tgt, 1e300)
    np.testing.assert_array_equal(big["xi"], big["used"])               # everything random is below


@pytest.mark.parametrize("pol", [(0, 0, 1.0), (1, 0, 1.0), (0, 1, 1.0), (1, 1, 1.0), (0, 2, 1.0), (1, 2, 1.0)])
@pytest.mark.parametrize("seed", range(3))
def test_alignment_under_every_policy(seed, pol):
    """S_{tau,sigma} on sigma equals R_{tau,sigma} on tau (map alignment) for
    every policy; positions P index S."""
    script = _with_policy(W.multiarea_p2p(P=4, n_e=40, n_i=10, k_e=8, k_i=2, k_remote_max=6, seed=70 + seed), pol)
    nets = [oracle.run_script(script, pl) for pl in range(4)]
    for sigma in range(4):
        s_off = nets[sigma].array("s_off").astype(np.int64)
        s_val = nets[sigma].array("s_val")
        for tau in range(4):
            r_off = nets[tau].array("r_off").astype(np.int64)
            np.testing.assert_array_equal(s_val[s_off[tau]:s_off[tau + 1]],
                                          nets[tau].array("r_val")[r_off[sigma]:r_off[sigma + 1]])
        tp = nets[sigma].array("tp_ptr").astype(np.int64)
        T, Pp = nets[sigma].array("t_val"), nets[sigma].array("p_val")
        for s in range(tp.size - 1):
            for tau, i in zip(T[tp[s]:tp[s + 1]], Pp[tp[s]:tp[s + 1]]):
                assert s_val[s_off[tau] + i] == s


@pytest.mark.parametrize("pol", [(0, 0, 1.0), (1, 0, 1.0), (1, 2, 1.0)])
def test_collective_i_holds_the_map_images(pol):
    script = _with_policy(W.balanced_collective(P=5, n_e=40, n_i=10, k_e=9, k_i=3), pol)
    for pl in range(5):
        net = oracle.run_script(script, pl)
        maps = _maps(net, 5)
        h_off = net.array("h_off").astype(np.int64)
        H, I = net.array("h_val"), net.array("i_val")
        for sigma in range(5):
            for j in range(h_off[sigma], h_off[sigma + 1]):
                want = maps.get((1, sigma, int(H[j])), -1) if sigma != pl else -1
                assert I[j] == want


def test_policy_arguments_checked():
    net = oracle.OracleNet(2, 0, 1, 0.1)
    for bad in ((2, 0, 1.0), (0, 3, 1.0), (-1, 0, 1.0), (0, 1, -0.5), (0, 1, float("nan"))):
        with pytest.raises(oracle.OracleError):
            net.set_map_policy(*bad)
    net.prepare()
    with pytest.raises(oracle.OracleError):
        net.set_map_policy(0, 0, 1.0)
