"""GPU parity of the map policies (images for used / all passed sources,
the threshold heuristic, images numbered canonically or in call order)
against the oracle, array by array."""
import numpy as np
import pytest

from gpu_util import compare_all, log
from paper_2512_09502_amd import workloads as W

pytestmark = pytest.mark.gpu

POLICIES = [(0, 0, 1.0), (1, 0, 1.0), (0, 1, 1.0), (1, 1, 1.0), (0, 2, 1.0), (1, 2, 1.0)]
CONST = {"weight": {"kind": "const", "mean": 1.0}, "delay": {"kind": "const", "mean": 1.0}}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


def _pol(script, pol):
    s = dict(script)
    s["map_policy"] = pol
    s["name"] = f"{script.get('name')}{pol}"
    return s


@pytest.mark.parametrize("pol", POLICIES[1:])
@pytest.mark.parametrize("seed", range(8))
def test_random_tiny_policies(seed, pol):
    s = _pol(W.random_tiny(500 + seed), pol)
    for pl in range(s["P"]):
        compare_all(s, pl)


@pytest.mark.parametrize("pol", [(1, 1, 1.0), (0, 2, 1.0), (1, 2, 1.0), (1, 0, 1.0)])
def test_multiarea_p2p_policies(pol):
    s = _pol(W.multiarea_p2p(P=6, n_e=800, n_i=200, k_e=40, k_i=10, k_remote_max=12), pol)
    for pl in (0, 5):
        n = compare_all(s, pl)
        log(f"multiarea {pol} P_local={pl}: {n} connections")


@pytest.mark.parametrize("pol", [(1, 0, 1.0), (1, 2, 1.0), (0, 1, 1.0)])
def test_collective_policies(pol):
    s = _pol(W.balanced_collective(P=12, n_e=400, n_i=100, k_e=90, k_i=22), pol)
    for pl in (0, 7):
        compare_all(s, pl)


THRESHOLD_CASES = [
    ({"rule": "fixed_indegree", "n": 9}, [(1, 0, 10)]),
    ({"rule": "fixed_indegree", "n": 10}, [(1, 0, 10)]),
    ({"rule": "pairwise_bernoulli", "p": 0.05}, [(1, 0, 10)]),
    ({"rule": "pairwise_bernoulli", "p": 0.2}, [(1, 0, 10)]),
    ({"rule": "fixed_total_number", "n": 50}, [(1, 0, 10)]),
    ({"rule": "fixed_total_number", "n": 150}, [(1, 0, 10)]),
    ({"rule": "fixed_outdegree", "n": 1}, [(1, 0, 10), (0, 0, 90)]),
    ({"rule": "one_to_one"}, [(1, 0, 10), (0, 0, 90)]),
    ({"rule": "assigned_nodes", "pairs": (list(range(50)), [i % 10 for i in range(50)])}, [(1, 0, 10)]),
    ({"rule": "assigned_nodes", "pairs": ([i % 60 for i in range(230)], [i % 10 if i < 30 else 10 + i % 90
                                                                          for i in range(230)])},
     [(1, 0, 10), (0, 0, 90)]),
]


@pytest.mark.parametrize("conn,tgt", THRESHOLD_CASES)
def test_threshold_cases(conn, tgt):
    b = W._Builder(2, seed=11)
    b.create(0, 100)
    b.create(1, 10)
    b.connect([(0, 0, 100)], tgt, conn, CONST, -1)
    s = _pol(b.script("xi_" + conn["rule"]), (1, 1, 1.0))
    for pl in (0, 1):
        compare_all(s, pl)


def test_images_without_connections():
    """All passed sources get images even where a call made no connection
    (in-degree 0, Bernoulli p = 0); the first-index array covers them."""
    b = W._Builder(3, seed=3)
    pops = [b.create(h, 50) for h in range(3)]
    b.connect(pops, pops, {"rule": "fixed_indegree", "n": 0}, CONST, -1)
    b.connect([pops[0], pops[2]], [pops[1]], {"rule": "pairwise_bernoulli", "p": 0.0}, CONST, 0)
    for pol in ((0, 2, 1.0), (1, 2, 1.0)):
        s = _pol(b.script("empty_calls"), pol)
        for pl in range(3):
            compare_all(s, pl)


def test_forced_map_path_matches_default():
    """The numbering-before-sort path under the default policy gives the
    oracle's default result (the same as the scan-after-sort path)."""
    import paper_2512_09502_amd as snnc
    import oracle
    from gpu_util import PREP_ARRAYS, compare
    s = W.random_tiny(7, P=3)
    for pl in range(3):
        net = snnc.run_script(s, pl, prepare=False, skip_invalid=True)
        net.tune("map_path", 1)
        net.prepare()
        ref = oracle.run_script(s, pl, skip_invalid=True)
        for k in PREP_ARRAYS:
            compare(k, net.array(k), ref.array(k), f"map_path P_local={pl}")
        net.close()


def test_policy_arguments_checked():
    import paper_2512_09502_amd as snnc
    net = snnc.Network(2, 0, 1, 0.1)
    for bad in ((2, 0, 1.0), (0, 3, 1.0), (-1, 0, 1.0), (0, 1, -0.5), (0, 1, float("nan")), (0, 1, float("inf"))):
        with pytest.raises(snnc.SnncError) as e:
            net.set_map_policy(*bad)
        assert e.value.code == -1
    net.prepare()
    with pytest.raises(snnc.SnncError) as e:
        net.set_map_policy(0, 0, 1.0)
    assert e.value.code == -4
    net.close()
