"""GPU parity of the assigned-nodes rule against the oracle: random pair
lists over multi-host segment sets under the map policies, the paper's
triplet procedure for a distributed fixed in-degree, the counting path under
a resident budget (targets on several hosts), and the argument checks."""
import numpy as np
import pytest

import oracle
from gpu_util import GEN_ARRAYS, PREP_ARRAYS, compare, compare_all, log
from paper_2512_09502_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


@pytest.mark.parametrize("seed", range(8))
def test_random_assigned(seed):
    s = W.random_assigned(seed)
    for pl in range(s["P"]):
        compare_all(s, pl)


@pytest.mark.parametrize("pol", [(1, 0, 1.0), (0, 1, 1.0), (1, 2, 1.0)])
@pytest.mark.parametrize("seed", range(3))
def test_random_assigned_policies(seed, pol):
    s = dict(W.random_assigned(60 + seed, P=3), map_policy=pol)
    for pl in range(3):
        compare_all(s, pl)


def test_distributed_indegree_by_triplets():
    s = W.distributed_indegree_assigned(P=4, n_per_host=3000, K=40, seed=7)
    for pl in (0, 3):
        n = compare_all(s, pl)
        log(f"  {n} connections on host {pl}")


def test_assigned_under_budget_counts_on_device():
    """Targets on several hosts: the local count needs a device pass (run on
    the counting stream when a resident budget is set)."""
    import paper_2512_09502_amd as snnc
    s = W.random_assigned(5, P=3)
    for pl in range(3):
        plain = snnc.run_script(s, pl, prepare=False)
        gen_a = {k: plain.array(k) for k in GEN_ARRAYS}
        plain.close()
        net = snnc.Network(s["P"], pl, s["seed"], s["dt"])
        net.set_resident_budget(1 << 30)
        for op in s["ops"]:
            if op[0] == "create":
                net.create(op[1], op[2])
            else:
                net.connect(*op[1:])
        for k in GEN_ARRAYS:
            np.testing.assert_array_equal(net.array(k), gen_a[k], err_msg=k)
        net.close()


def test_assigned_argument_checks():
    import paper_2512_09502_amd as snnc
    syn = {"weight": {"kind": "const", "mean": 1.0}, "delay": {"kind": "const", "mean": 1.0}}
    net = snnc.Network(1, 0, 1, 0.1)
    net.create(0, 10)
    for ps, pt in (([5], [0]), ([0], [10])):
        with pytest.raises(snnc.SnncError) as e:
            net.connect_assigned([(0, 0, 5)], [(0, 0, 10)], ps, pt, syn)
        assert e.value.code == -1
    with pytest.raises(snnc.SnncError) as e:
        net.connect([(0, 0, 5)], [(0, 0, 10)], {"rule": "assigned_nodes", "pairs": ([0, 1], [0])}, syn)
    assert e.value.code == -1
    for entry in ("snnc_connect", "snnc_submit"):
        with pytest.raises(snnc.SnncError) as e:
            net._connect_like(entry, [(0, 0, 5)], [(0, 0, 10)], {"rule": "assigned_nodes", "n": 0}, syn, -1)
        assert e.value.code == -1
    cid = net.connect_assigned([(0, 0, 5)], [(0, 0, 10)], [], [], syn)      # no pairs: an empty call
    net.prepare()
    assert net.count("src") == 0
    net.close()
