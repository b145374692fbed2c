"""The allocation-free sort entry point (snnc_sort_pairs_noalloc) through the
C ABI against snnc_sort_pairs on the same inputs: identical sorted keys and
payloads, bit for bit, on two calls in a row (the second smaller, so the
static scratch keeps the first call's contents), with no device allocation by
the library during the calls; sizes above the scratch's limit are refused."""
import numpy as np
import pytest

import paper_2512_09502_amd as snnc
from gpu_util import log

pytestmark = pytest.mark.gpu


def _keys(torch, n, bits, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    k = torch.randint(0, 1 << bits, (n,), generator=g, dtype=torch.int64) << 16
    v = torch.arange(n, dtype=torch.int32)
    return k.cuda(), v.cuda()


def _ref(net, torch, k, v, lo, hi):
    kk, vv = net.sort_pairs(k.clone(), v.clone(), lo, hi)
    return kk.cpu().numpy(), vv.cpu().numpy()


@pytest.mark.parametrize("sizes", [(3_000_001, 777_777), (9_000_000, 65_536), (200_000, 1)])
def test_noalloc_sort_equals_sort_pairs(sizes):
    import torch
    torch.cuda.set_device(0)
    net = snnc.Network(1, 0, 1, 0.1)
    for call, (n, bits) in enumerate(zip(sizes, (34, 21))):
        k, v = _keys(torch, n, bits, 100 + call)
        want_k, want_v = _ref(net, torch, k, v, 16, 16 + bits)
        kt, vt = torch.empty_like(k), torch.empty_like(v)
        torch.cuda.synchronize()
        before = net.stats()
        got_k, got_v = net.sort_pairs_noalloc(k, v, kt, vt, 16, 16 + bits)
        after = net.stats()
        assert after["bytes_live"] == before["bytes_live"] and after["bytes_peak"] == before["bytes_peak"]
        np.testing.assert_array_equal(got_k.cpu().numpy(), want_k)
        np.testing.assert_array_equal(got_v.cpu().numpy(), want_v)
        log(f"noalloc sort call {call}: {n} pairs, {bits} bits equal snnc_sort_pairs")
    net.close()


def test_noalloc_sort_refuses_sizes_above_the_scratch():
    import torch
    torch.cuda.set_device(0)
    net = snnc.Network(1, 0, 1, 0.1)
    n = 80_000_000            # look-back table of 80e6 / 8192 tiles x 512 buckets x 8 B > 16 MiB
    k = torch.empty(n, dtype=torch.int64, device="cuda")
    v = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(snnc.SnncError) as e:
        net.sort_pairs_noalloc(k, v, torch.empty_like(k), torch.empty_like(v), 16, 16 + 40)
    assert e.value.code == -1 and "static scratch" in str(e.value)
    # the context still works afterwards
    k2, v2 = _keys(torch, 1000, 20, 5)
    kk, vv = net.sort_pairs_noalloc(k2, v2, torch.empty_like(k2), torch.empty_like(v2), 16, 36)
    assert bool((kk[1:] >= kk[:-1]).all())
    net.close()
