"""Pins of the GPU memory levels in the oracle (Methods, GPU memory levels
subsection): level 0 gives images to the used remote sources, levels 1 to 3
to every passed source; levels 0 and 1 keep the first index and count of each
image row apart from the first-index array of the local rows, level 3 keeps
the counts beside it.  The row arrays are checked against the sorted
connections themselves (first position and multiplicity of each image
source), and delivery gives the same events at every level with the same
images."""
import numpy as np
import pytest

import oracle
from paper_2512_09502_amd import workloads as W


def _script(level=None, pol=None):
    s = W.multiarea_p2p(P=4, n_e=40, n_i=10, k_e=8, k_i=2, k_remote_max=6, seed=71)
    s = dict(s)
    if level is not None:
        s["memory_level"] = level
    if pol is not None:
        s["map_policy"] = pol
    return s


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_image_rows_per_level(level):
    for pl in (0, 2):
        net = oracle.run_script(_script(level), pl)
        M = net.neurons(pl)
        src = net.array("src").astype(np.int64)
        n_img = net.array("r_val").size
        counts = np.bincount(src, minlength=M + n_img)
        firsts = np.searchsorted(src, np.arange(M + n_img))          # sorted by source first
        rp = net.array("row_ptr")
        if level in (0, 1):
            assert rp.size == M + 1
            np.testing.assert_array_equal(rp, firsts[:M].tolist() + [firsts[M] if n_img else src.size])
            np.testing.assert_array_equal(net.array("img_first"), firsts[M:])
        else:
            assert rp.size == M + n_img + 1
            np.testing.assert_array_equal(np.diff(rp.astype(np.int64)), counts)
            with pytest.raises(oracle.OracleError):
                net.array("img_first")
        if level == 2:
            with pytest.raises(oracle.OracleError):
                net.array("img_count")
        else:
            np.testing.assert_array_equal(net.array("img_count"), counts[M:])


def test_level_sets_the_image_sources():
    for pl in (1, 3):
        used = oracle.run_script(_script(pol=(0, 0, 1.0)), pl).array("r_val")
        allp = oracle.run_script(_script(pol=(0, 2, 1.0)), pl).array("r_val")
        assert used.size < allp.size
        np.testing.assert_array_equal(oracle.run_script(_script(0), pl).array("r_val"), used)
        for level in (1, 2, 3):
            np.testing.assert_array_equal(oracle.run_script(_script(level), pl).array("r_val"), allp)
        # a map policy set after the level decides the image sources
        np.testing.assert_array_equal(oracle.run_script(_script(1, pol=(0, 0, 1.0)), pl).array("r_val"), used)


def test_delivery_equal_across_levels():
    rng = np.random.default_rng(2)
    pl = 1
    outs = []
    for level in (1, 2, 3):
        net = oracle.run_script(_script(level), pl)
        r_off = net.array("r_off").astype(np.int64)
        host, pos = [], []
        for sigma in range(4):
            if sigma == pl:
                continue
            k = int(r_off[sigma + 1] - r_off[sigma])
            sel = np.random.default_rng(sigma).permutation(k)[:30]
            host += [sigma] * sel.size
            pos += sel.tolist()
        mult = rng.integers(1, 4, size=len(host))
        outs.append(net.deliver(0, host, pos, mult))
        rng = np.random.default_rng(2)
    for o in outs[1:]:
        for k in outs[0]:
            np.testing.assert_array_equal(o[k], outs[0][k], err_msg=k)


def test_level_arguments():
    net = oracle.OracleNet(2, 0, 1, 0.1)
    with pytest.raises(oracle.OracleError):
        net.set_memory_level(4)
    with pytest.raises(oracle.OracleError):
        net.set_memory_level(-1)
    net.set_memory_level(0)
    net.prepare()
    with pytest.raises(oracle.OracleError):
        net.set_memory_level(1)
