"""Pins of the oracle's spike exchange through the built maps (Appendix E:
packet and delivery figures; collective subsection): the worked example as
printed, and end to end on random multi-host networks -- a spike of neuron s
on host sigma, packed on sigma and delivered on tau, yields exactly tau's
connections whose source is (sigma, s), found from tau's generation records
without the maps."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2512_09502_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _app_e_lists():
    """T/P lists of source host 0 with the App. E positions (other list
    entries filled with increasing ids, as the maps are sorted)."""
    g = json.load(open(os.path.join(GOLDEN, "app_e_send_tables.json")))
    P, M = g["P"], 800
    lists = []
    for tau in range(P):
        pos = {int(s): p for s, p in g["positions"].get(str(tau), {}).items()}
        n = (max(pos.values()) + 1) if pos else 0
        free = [x for x in range(M) if x not in pos]
        lst = []
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
        lists.append(lst)
    ptr, which, where = oracle.transpose_lists(lists, M)
    return P, M, ptr, which, where


def test_app_e_packets():
    """Neurons 480 and 742 of rank 0 spike: the packet for rank 1 holds the
    positions 127 and 271, the packet for rank 2 holds 113."""
    P, M, ptr, which, where = _app_e_lists()
    out = oracle.packets_from_lists(ptr, which, where, M, P, [480, 742], [2, 3])
    off = out["off"].astype(np.int64)
    assert off.tolist() == [0, 0, 2, 3]
    assert out["pos"][off[1]:off[2]].tolist() == [127, 271]
    assert out["pos"][off[2]:off[3]].tolist() == [113]
    assert out["mult"].tolist() == [2, 3, 3]
    # spike order decides the order inside a packet
    out2 = oracle.packets_from_lists(ptr, which, where, M, P, [742, 480])
    assert out2["pos"][:2].tolist() == [271, 127]


def test_app_e_delivery():
    """Rank 1 receives positions 127 and 271 from rank 0; reading of the
    figure: they map to the images 357 and 698 in that order.  Image 357 has
    connections to 126 (delay 2) and 308 (delay 5), image 698 to 243 (delay 3)."""
    g = json.load(open(os.path.join(GOLDEN, "app_e_delivery_blocks.json")))
    c = np.array(g["connections"])
    w = np.array([0.5, 0.25, 2.0], np.float32)
    csr = oracle.sort_csr(c[:, 0], c[:, 1], c[:, 2], w, 1000)
    img = np.full(272, -1, np.int32)
    img[127], img[271] = 357, 698
    out = oracle.deliver_from_maps([0, 272], img, csr["row_ptr"], csr["tgt"], csr["delay"], csr["weight"],
                                   [0, 0], [127, 271], [1, 4])
    assert out["image"].tolist() == [357, 698]
    assert out["tgt"].tolist() == [126, 308, 243]
    assert out["delay"].tolist() == [2, 5, 3]
    assert out["weight"].tolist() == [2.0, 0.25, 0.5 * 4]        # weight x multiplicity
    rb, re = out["row_begin"].astype(np.int64), out["row_end"].astype(np.int64)
    assert (re - rb).tolist() == [2, 1]


def _origin_records(script, net, pl):
    """Generation records of host pl with the original source (host, local id)."""
    rejected = {k for k, _ in net.rejected}
    ops = [op for k, op in enumerate(script["ops"]) if op[0] == "connect" and k not in rejected]
    off = net.array("call_off").astype(np.int64)
    gs, gt = net.array("gen_src"), net.array("gen_tgt")
    gd, gw = net.array("gen_delay"), net.array("gen_weight")
    recs = []
    for c, op in enumerate(ops):
        for i in range(off[c], off[c + 1]):
            o = int(gs[i])
            for h, f, n in op[1]:
                if o < n:
                    recs.append((h, f + o, int(gt[i]), int(gd[i]), float(gw[i]), i))
                    break
                o -= n
    return recs


def _expected_events(recs, sigma, spikes, mult):
    """Connections from (sigma, s) for each spike, in (target, generation) order."""
    ev = []
    for s, m in zip(spikes, mult):
        mine = sorted([r for r in recs if r[0] == sigma and r[1] == s], key=lambda r: (r[2], r[5]))
        ev += [(r[2], r[3], float(np.float32(r[4]) * np.float32(m))) for r in mine]
    return ev


@pytest.mark.parametrize("pol", [None, (1, 2, 1.0), (1, 1, 1.0)])
@pytest.mark.parametrize("seed", range(3))
def test_point_to_point_round_trip(seed, pol):
    script = W.multiarea_p2p(P=4, n_e=40, n_i=10, k_e=8, k_i=2, k_remote_max=6, seed=90 + seed)
    if pol is not None:
        script = dict(script, map_policy=pol)
    P = script["P"]
    nets = [oracle.run_script(script, pl) for pl in range(P)]
    recs = [_origin_records(script, nets[pl], pl) for pl in range(P)]
    rng = np.random.default_rng(seed)
    for sigma in range(P):
        M = nets[sigma].neurons(sigma)
        spikes = rng.choice(M, size=12, replace=False)
        mult = rng.integers(1, 4, size=12)
        pk = nets[sigma].spike_packets(0, spikes, mult)
        off = pk["off"].astype(np.int64)
        assert off[sigma + 1] == off[sigma]                       # nothing for the own host
        for tau in range(P):
            if tau == sigma:
                continue
            pos, m = pk["pos"][off[tau]:off[tau + 1]], pk["mult"][off[tau]:off[tau + 1]]
            r_off = nets[tau].array("r_off").astype(np.int64)
            R = nets[tau].array("r_val")[r_off[sigma]:r_off[sigma + 1]]
            sent = R[pos]                                         # the map entries name the spiking neurons
            order = [int(s) for s in spikes if int(s) in set(R.tolist())]
            assert sent.tolist() == order
            d = nets[tau].deliver(0, np.full(len(pos), sigma), pos, m)
            got = list(zip(d["tgt"].tolist(), d["delay"].tolist(), d["weight"].tolist()))
            mult_of = dict(zip(spikes.tolist(), mult.tolist()))
            assert got == _expected_events(recs[tau], sigma, order, [mult_of[s] for s in order])


@pytest.mark.parametrize("pol", [None, (1, 0, 1.0)])
def test_collective_round_trip(pol):
    script = W.balanced_collective(P=4, n_e=40, n_i=10, k_e=6, k_i=2)
    if pol is not None:
        script = dict(script, map_policy=pol)
    P = script["P"]
    nets = [oracle.run_script(script, pl) for pl in range(P)]
    recs = [_origin_records(script, nets[pl], pl) for pl in range(P)]
    rng = np.random.default_rng(3)
    for sigma in range(P):
        spikes = rng.choice(nets[sigma].neurons(sigma), size=10, replace=False)
        pk = nets[sigma].spike_packets(1, spikes)
        off = pk["off"].astype(np.int64)
        assert off.tolist() == [0, 10]                            # one group, every neuron reports to it
        h_off = nets[sigma].array("h_off").astype(np.int64)
        H = nets[sigma].array("h_val")[h_off[sigma]:h_off[sigma + 1]]
        assert H[pk["pos"]].tolist() == spikes.tolist()           # Q indexes H_{0, sigma}
        for tau in range(P):
            if tau == sigma:
                continue
            d = nets[tau].deliver(1, np.full(10, sigma), pk["pos"], pk["mult"], grp=np.zeros(10))
            got = list(zip(d["tgt"].tolist(), d["delay"].tolist(), d["weight"].tolist()))
            assert got == _expected_events(recs[tau], sigma, spikes.tolist(), [1] * 10)
            has = [any(r[0] == sigma and r[1] == s for r in recs[tau]) for s in spikes]
            assert ((d["image"] >= 0) == np.array(has)).all()    # -1 exactly for sources without an image


def test_spike_exchange_errors():
    script = W.multiarea_p2p(P=3, n_e=20, n_i=5, k_e=4, k_i=1, k_remote_max=4, seed=5)
    net = oracle.run_script(script, 0)
    with pytest.raises(oracle.OracleError):
        net.spike_packets(0, [net.neurons(0)])                    # not a local neuron
    with pytest.raises(oracle.OracleError):
        net.deliver(0, [0], [0])                                  # own host has no map
    n1 = int(net.array("r_off")[2] - net.array("r_off")[1])
    with pytest.raises(oracle.OracleError):
        net.deliver(0, [1], [n1])                                 # beyond the map
