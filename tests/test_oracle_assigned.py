"""Pins of the oracle's assigned-nodes rule (Methods, distributed fixed
in-degree subsection: the triplets drawn on a target host are sorted by
source host and position and connected with a rule that takes source and
target as given).  Each pair lands exactly once, on its target's host, with
element index = pair index; a pair list (i, i) reproduces one-to-one
including the synapse values; the paper's triplet procedure gives every
target exactly K connections; the union of the hosts' shares equals the
one-host build; the point-to-point maps stay aligned."""
import numpy as np
import pytest

import oracle
from paper_2512_09502_amd import workloads as W
from test_oracle_maps import _flatten_to_one_host, _records, _sorted_concat

SYN = {"weight": {"kind": "normal", "mean": 0.2, "sd": 0.05},
       "delay": {"kind": "normal", "mean": 1.5, "sd": 0.5, "lo": 0.1}}


def _set_lookup(segs, ordinal):
    for h, f, n in segs:
        if ordinal < n:
            return h, f + ordinal
        ordinal -= n
    raise AssertionError


@pytest.mark.parametrize("seed", range(10))
def test_pairs_land_on_their_target_host(seed):
    script = W.random_assigned(seed)
    P = script["P"]
    ops = [op for op in script["ops"] if op[0] == "connect"]
    for pl in range(P):
        net = oracle.run_script(script, pl)
        off = net.array("call_off").astype(np.int64)
        gs, gt, ge = net.array("gen_src"), net.array("gen_tgt"), net.array("gen_e")
        for c, op in enumerate(ops):
            _, src, tgt, conn, syn, alpha = op
            if conn["rule"] != "assigned_nodes":
                continue
            ps, pt = conn["pairs"]
            want = [(int(s), _set_lookup(tgt, int(t))[1], i) for i, (s, t) in enumerate(zip(ps, pt))
                    if _set_lookup(tgt, int(t))[0] == pl]
            got = list(zip(gs[off[c]:off[c + 1]].tolist(), gt[off[c]:off[c + 1]].tolist(),
                           ge[off[c]:off[c + 1]].tolist()))
            assert got == want


def test_diagonal_pairs_reproduce_one_to_one():
    """Pairs (i, i) are the one-to-one rule: same positions, same element
    index, hence the same synapse draws (independent branches of the oracle)."""
    out = []
    for conn in ({"rule": "one_to_one"}, {"rule": "assigned_nodes", "pairs": (list(range(37)), list(range(37)))}):
        b = W._Builder(2, seed=5)
        a = b.create(0, 30)
        c = b.create(1, 30)
        b.connect([(0, 3, 20), (1, 0, 17)], [(1, 5, 25), (0, 0, 12)], conn, SYN)
        script = b.script("diag")
        out.append([oracle.run_script(script, pl) for pl in range(2)])
    for pl in range(2):
        for k in ("gen_src", "gen_tgt", "gen_e", "gen_delay", "gen_weight", "src", "tgt", "row_ptr"):
            np.testing.assert_array_equal(out[0][pl].array(k), out[1][pl].array(k), err_msg=k)


def test_triplet_procedure_gives_exact_indegree():
    script = W.distributed_indegree_assigned(P=3, n_per_host=40, K=9, seed=3)
    for pl in range(3):
        net = oracle.run_script(script, pl)
        counts = np.bincount(net.array("gen_tgt"), minlength=40)
        assert (counts == 9).all()                           # K per target, from all source hosts
        # the calls of one target host carry sources sorted by (sigma, s)
    ops = [op for op in script["ops"] if op[0] == "connect"]
    assert len(ops) == 9
    for op in ops:
        s = np.asarray(op[3]["pairs"][0])
        assert (np.diff(s) >= 0).all()


@pytest.mark.parametrize("seed", range(8))
def test_union_of_shares_equals_one_host_build(seed):
    script = W.random_assigned(40 + seed, P=int(2 + seed % 3))
    P = script["P"]
    shares = [oracle.run_script(script, pl) for pl in range(P)]
    flat, remap_seg = _flatten_to_one_host(script)
    one = oracle.run_script(flat, 0)
    recs = [_records(sh, lambda t, pl=pl: remap_seg(pl, t, 1)[0][1]) for pl, sh in enumerate(shares)]
    a = _sorted_concat(recs)
    b = _sorted_concat([_records(one, lambda t: t)])
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("pol", [None, (1, 1, 1.0), (0, 2, 1.0)])
@pytest.mark.parametrize("seed", range(4))
def test_p2p_alignment_with_assigned_calls(seed, pol):
    script = W.random_assigned(80 + seed, P=3)
    if pol is not None:
        script = dict(script, map_policy=pol)
    nets = [oracle.run_script(script, pl) for pl in range(3)]
    for sigma in range(3):
        s_off = nets[sigma].array("s_off").astype(np.int64)
        s_val = nets[sigma].array("s_val")
        for tau in range(3):
            r_off = nets[tau].array("r_off").astype(np.int64)
            np.testing.assert_array_equal(s_val[s_off[tau]:s_off[tau + 1]],
                                          nets[tau].array("r_val")[r_off[sigma]:r_off[sigma + 1]])


def test_assigned_errors():
    b = W._Builder(1, seed=1)
    b.create(0, 10)
    net = oracle.OracleNet(1, 0, 1, 0.1)
    net.create(0, 10)
    with pytest.raises(oracle.OracleError):
        net.connect([(0, 0, 5)], [(0, 0, 10)], {"rule": "assigned_nodes", "pairs": ([5], [0])}, SYN)   # source 5 of 5
    with pytest.raises(oracle.OracleError):
        net.connect([(0, 0, 5)], [(0, 0, 10)], {"rule": "assigned_nodes", "pairs": ([0], [10])}, SYN)
    with pytest.raises(oracle.OracleError):
        net.connect([(0, 0, 5)], [(0, 0, 10)], {"rule": "assigned_nodes", "pairs": ([0, 1], [0])}, SYN)
    with pytest.raises(oracle.OracleError):
        net._conn(oracle.lib().orc_connect, [(0, 0, 5)], [(0, 0, 10)], {"rule": "assigned_nodes", "n": 1}, SYN, -1)
    net.connect([(0, 0, 5)], [(0, 0, 10)], {"rule": "assigned_nodes", "pairs": ([], [])}, SYN)        # empty is fine
    assert net.array("gen_src").size == 0
