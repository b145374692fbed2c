"""GPU parity of the GPU memory levels: every array equals the oracle's at
each level (point-to-point and collective layouts), the arrays that levels 0
and 1 keep in host memory are host-resident and readable by the delivery
kernels, and the device holds fewer bytes at level 1 than at level 2."""
import numpy as np
import pytest

import oracle
from gpu_util import compare_all, log
from paper_2512_09502_amd import workloads as W

pytestmark = pytest.mark.gpu

HOST_ARRAYS = ["r_off", "r_val", "img_base", "l_val", "h_off", "h_val", "i_val", "img_first", "img_count"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


def _p2p(level):
    return dict(W.multiarea_p2p(P=6, n_e=800, n_i=200, k_e=40, k_i=10, k_remote_max=12, seed=21), memory_level=level)


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_levels_point_to_point(level):
    for pl in (0, 4):
        compare_all(_p2p(level), pl)


@pytest.mark.parametrize("level", [0, 1, 3])
def test_levels_collective(level):
    s = dict(W.balanced_collective(P=12, n_e=400, n_i=100, k_e=90, k_i=22), memory_level=level)
    for pl in (0, 7):
        compare_all(s, pl)


@pytest.mark.parametrize("level", [1, 2])
def test_placement_and_delivery(level):
    import paper_2512_09502_amd as snnc
    from test_spikes_gpu import _check_deliver
    s = _p2p(level)
    pl = 2
    net = snnc.run_script(s, pl)
    ref = oracle.run_script(s, pl)
    for k in HOST_ARRAYS:
        try:
            where = net.on_host(k)
        except snnc.SnncError:
            continue                      # not kept at this level
        assert where == (level <= 1), k
    assert not net.on_host("row_ptr") and not net.on_host("src")
    rng = np.random.default_rng(5)
    r_off = ref.array("r_off").astype(np.int64)
    host, pos = [], []
    for sigma in range(6):
        if sigma == pl:
            continue
        k = int(r_off[sigma + 1] - r_off[sigma])
        sel = rng.permutation(k)[: min(k, 300)]
        host += [sigma] * sel.size
        pos += sel.tolist()
    ref_ev = _check_deliver(net, ref, 0, host, pos, rng.integers(1, 5, size=len(host)))
    log(f"level {level}: {len(host)} entries, {ref_ev['tgt'].size} events")
    net.close()


def test_device_bytes_by_level():
    """~2.8e5 images per host: maps and image rows of several MB leave the device at level 1."""
    import paper_2512_09502_amd as snnc
    live = {}
    big = W.multiarea_p2p(P=8, n_e=40000, n_i=10000, k_e=40, k_i=10, k_remote_max=30, seed=3)
    for level in (1, 2):
        net = snnc.run_script(dict(big, memory_level=level), 1)
        net.sync()
        live[level] = net.stats()["bytes_live"]
        net.close()
    log(f"device bytes after prepare: level 1 {live[1]}, level 2 {live[2]}")
    assert live[1] < live[2]
