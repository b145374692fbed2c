"""GPU checks of the radix sort on its own: every tile-shape variant against
numpy's stable argsort on random keys (ragged sizes, narrow and wide bit
ranges, many equal keys)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def net():
    import torch
    import paper_2512_09502_amd as snnc
    torch.cuda.set_device(0)
    n = snnc.Network(1, 0, 1, 0.1)
    yield n
    n.close()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("variant", range(14))
@pytest.mark.parametrize("n,lo,hi", [(1, 0, 8), (4095, 16, 50), (100003, 16, 50), (333333, 0, 64), (77777, 3, 9),
                                     (250000, 16, 20)])
def test_sort_pairs_matches_stable_argsort(net, mode, variant, n, lo, hi):
    import torch
    net.tune("digit_bits", 0)
    net.tune("sort_mode", mode)
    rng = np.random.default_rng(n + variant + 31 * lo)
    keys = rng.integers(0, 2**63, size=n, dtype=np.int64).view(np.uint64)
    if hi - lo <= 8:
        keys &= np.uint64(((1 << 64) - 1) ^ (((1 << 4) - 1) << lo))    # only half the digit values: many ties
    vals = np.arange(n, dtype=np.int32)
    net.tune("sort_variant", variant)
    k, v = net.sort_pairs(torch.from_numpy(keys.view(np.int64)).cuda(), torch.from_numpy(vals).cuda(), lo, hi)
    mask = np.uint64(((1 << (hi - lo)) - 1) << lo) if hi - lo < 64 else np.uint64((1 << 64) - 1)
    order = np.argsort(keys & mask, kind="stable")
    np.testing.assert_array_equal(v.cpu().numpy(), order.astype(np.int32))
    np.testing.assert_array_equal(k.cpu().numpy().view(np.uint64), keys[order])


def test_autotune_picks_a_valid_setting_and_caches_it(net):
    import torch
    r = net.autotune_sort(200003, 30)
    assert r["sort_mode"] in (0, 1) and 0 <= r["sort_variant"] < 14 and r["ms"] > 0
    again = net.autotune_sort(200003 + 5, 30)        # same size class: served from the cache
    assert (again["sort_mode"], again["sort_variant"]) == (r["sort_mode"], r["sort_variant"]) and again["ms"] == -1
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 2**46, size=200003, dtype=np.int64).view(np.uint64)
    vals = np.arange(keys.size, dtype=np.int32)
    k, v = net.sort_pairs(torch.from_numpy(keys.view(np.int64)).cuda(), torch.from_numpy(vals).cuda(), 16, 46)
    order = np.argsort(keys >> np.uint64(16), kind="stable")
    np.testing.assert_array_equal(v.cpu().numpy(), order.astype(np.int32))


@pytest.mark.parametrize("digit_bits", [8, 9])
@pytest.mark.parametrize("variant", [0, 2, 3, 6, 7, 8, 9])
@pytest.mark.parametrize("n,lo,hi", [(8193, 16, 50), (300007, 16, 43), (65536, 0, 64), (5000, 7, 16), (1, 16, 25)])
def test_digit_width(net, digit_bits, variant, n, lo, hi):
    """8- and 9-bit digits (256 / 512 buckets) give the same stable order."""
    import torch
    net.tune("sort_mode", 0)
    net.tune("sort_variant", variant)
    net.tune("digit_bits", digit_bits)
    rng = np.random.default_rng(n + 7 * variant + digit_bits)
    keys = rng.integers(0, 2**63, size=n, dtype=np.int64).view(np.uint64)
    keys[::3] = keys[0]                                   # long runs of equal keys
    vals = np.arange(n, dtype=np.int32)
    k, v = net.sort_pairs(torch.from_numpy(keys.view(np.int64)).cuda(), torch.from_numpy(vals).cuda(), lo, hi)
    mask = np.uint64(((1 << (hi - lo)) - 1) << lo) if hi - lo < 64 else np.uint64((1 << 64) - 1)
    order = np.argsort(keys & mask, kind="stable")
    np.testing.assert_array_equal(v.cpu().numpy(), order.astype(np.int32))
    np.testing.assert_array_equal(k.cpu().numpy().view(np.uint64), keys[order])
    net.tune("digit_bits", 0)
