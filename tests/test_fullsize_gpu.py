"""Parity at the benchmark's full sizes, in the same launch configuration.

The oracle cannot build 4e8-2.25e9 connections in test time, so:
  * generation order: sampled elements of every call are recomputed one by
    one by the oracle (independent-element rules) and compared exactly;
  * after Prepare, properties that hold at any size are checked on the GPU
    with torch (an implementation independent of the library): source-major
    order, first-index array = histogram of the sources, the sorted network is
    the same multiset as the generated one (modular hash sums), the image map
    equals the set of used remote sources (scatter bitmap), the collective I
    array matches that bitmap, and point-to-point sequences on the source host
    equal the maps on two target hosts.
"""
import numpy as np
import pytest

import oracle
import paper_2512_09502_amd as snnc
from gpu_util import log, ulp_diff
from paper_2512_09502_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

MOD = 2147483647          # 2^31 - 1
CHUNK = 1 << 27


def _torch():
    import torch
    torch.cuda.set_device(0)
    return torch


def _build(script, P_local):
    net = snnc.Network(script["P"], P_local, script["seed"], script["dt"])
    for op in script["ops"]:
        if op[0] == "create":
            net.create(op[1], op[2])
        else:
            _, src, tgt, conn, syn, alpha = op
            net.connect(src, tgt, conn, syn, alpha)
    return net


def _sample_generation(net, ref, n_samples=400, seed=0):
    """Sampled positions of the generation-order arrays against the oracle's
    element-by-element recomputation; position - call start = element index
    for these workloads (local targets first in every target set)."""
    off = net.array("call_off").astype(np.int64)
    rng = np.random.default_rng(seed)
    pos = np.unique(np.concatenate([rng.integers(0, off[-1], size=n_samples), off[:-1][np.diff(off) > 0],
                                    off[1:][np.diff(off) > 0] - 1]))
    bad = 0
    for p in pos:
        c = int(np.searchsorted(off, p, side="right") - 1)
        e = int(p - off[c])
        r = ref.element(c, e)
        got = {k: net.array_range("gen_" + k, int(p), 1)[0] for k in ("src", "tgt", "delay", "weight")}
        assert r is not None
        ok = (got["src"] == r["src"] and got["tgt"] == r["tgt"] and got["delay"] == r["delay"]
              and ulp_diff(np.array([got["weight"]], np.float32), np.array([r["weight"]], np.float32)) <= 2)
        bad += not ok
        assert ok, f"position {p} (call {c}, element {e}): {got} vs oracle {r}"
    return len(pos)


def _hash(torch, src, tgt, delay, wbits):
    h = (src.long() * 1000003 + tgt.long()) % MOD
    h = (h * 1000033 + delay.long()) % MOD
    h = (h * 999983 + (wbits.long() & 0x7FFFFFFF)) % MOD
    return h


def _hash_sums(torch, src_fn, tgt, delay, weight, n):
    s1 = torch.zeros((), dtype=torch.int64, device="cuda")
    s2 = torch.zeros((), dtype=torch.int64, device="cuda")
    for a in range(0, n, CHUNK):
        b = min(n, a + CHUNK)
        h = _hash(torch, src_fn(a, b), tgt[a:b], delay[a:b], weight[a:b].view(torch.int32))
        s1 += h.sum()
        s2 += ((h * 48271) % MOD).sum()
    return int(s1), int(s2)


def _check_sorted_and_csr(torch, src, tgt, row_ptr, n):
    for a in range(0, n, CHUNK):
        b = min(n, a + CHUNK + 1)
        k = src[a:b].long() * (1 << 32) + tgt[a:b].long()
        assert bool((k[1:] >= k[:-1]).all()), f"not source-major near {a}"
    rp = row_ptr
    assert int(rp[0]) == 0 and int(rp[-1]) == n
    counts = torch.bincount(src.long(), minlength=rp.numel() - 1)
    assert torch.equal(counts, rp[1:] - rp[:-1])


def test_column8_full_size():
    torch = _torch()
    script = W.column8()
    net = _build(script, 0)
    ref = oracle.run_script(script, 0, declare_only=True)
    k = _sample_generation(net, ref)
    log(f"column8 full: {k} sampled elements equal the oracle")
    # generated connections as (source local id, target, delay, weight)
    n = net.count("gen_src")
    off = net.array("call_off").astype(np.int64)
    first = np.array([op[1][0][1] for op in script["ops"] if op[0] == "connect"], np.int64)   # one source segment
    call_first = torch.from_numpy(np.repeat(first, np.diff(off))).cuda()
    g_src, g_tgt = net.tensor("gen_src"), net.tensor("gen_tgt")
    g_delay, g_w = net.tensor("gen_delay"), net.tensor("gen_weight")
    before = _hash_sums(torch, lambda a, b: g_src[a:b].long() + call_first[a:b], g_tgt, g_delay, g_w, n)
    del call_first, g_src, g_tgt, g_delay, g_w
    net.prepare()
    src, tgt, rp = net.tensor("src"), net.tensor("tgt"), net.tensor("row_ptr")
    _check_sorted_and_csr(torch, src, tgt, rp, n)
    after = _hash_sums(torch, lambda a, b: src[a:b], tgt, net.tensor("delay"), net.tensor("weight"), n)
    assert before == after, "sorted network is not the generated multiset"
    net.close()


def _global_prefix_of_gen(torch, net, script, P_local):
    """For the generated connections: global source prefix (alpha+1) G + gid, or
    -1 - local id for sources on P_local."""
    P = script["P"]
    M = [0] * P
    for op in script["ops"]:
        if op[0] == "create":
            M[op[1]] += op[2]
    base = np.concatenate([[0], np.cumsum(M)]).astype(np.int64)
    G = int(base[-1])
    calls = [op for op in script["ops"] if op[0] == "connect"]
    off = net.array("call_off").astype(np.int64)
    out = torch.empty(int(off[-1]), dtype=torch.int64, device="cuda")
    g_src = net.tensor("gen_src")
    for c, op in enumerate(calls):
        a, b = int(off[c]), int(off[c + 1])
        if a == b:
            continue
        segs = op[1]
        ordb = np.concatenate([[0], np.cumsum([s[2] for s in segs])]).astype(np.int64)
        ords = g_src[a:b].long()
        seg_idx = torch.searchsorted(torch.from_numpy(ordb[1:]).cuda(), ords, right=True)
        hosts = torch.tensor([s[0] for s in segs], device="cuda")[seg_idx]
        firsts = torch.tensor([s[1] for s in segs], device="cuda", dtype=torch.int64)[seg_idx]
        local = firsts + ords - torch.from_numpy(ordb[:-1]).cuda()[seg_idx]
        gid = torch.from_numpy(base[:-1]).cuda()[hosts] + local
        pref = (op[5] + 1) * G + gid
        out[a:b] = torch.where(hosts == P_local, -1 - local, pref)
    return out, base, G


def test_collective_full_size():
    torch = _torch()
    script = W.balanced_collective()
    P, PL = script["P"], 0
    net = _build(script, PL)
    ref = oracle.run_script(script, PL, declare_only=True)
    k = _sample_generation(net, ref, n_samples=300)
    log(f"collective full: {k} sampled elements equal the oracle")
    n = net.count("gen_src")
    pref, base, G = _global_prefix_of_gen(torch, net, script, PL)
    M_local = int(base[PL + 1] - base[PL])
    # the image map: used remote prefixes, by a scatter bitmap (torch)
    n_a = 2
    used = torch.zeros(n_a * G, dtype=torch.uint8, device="cuda")
    for a in range(0, n, CHUNK):
        p = pref[a:a + CHUNK]
        used[p[p >= 0]] = 1
    used_idx = torch.nonzero(used).flatten()
    g_tgt, g_delay, g_w = net.tensor("gen_tgt"), net.tensor("gen_delay"), net.tensor("gen_weight")
    # expected source' of each generated connection: local id or M_local + rank of its prefix
    rank = torch.cumsum(used.to(torch.int64), 0) - 1
    before = _hash_sums(torch, lambda a, b: torch.where(pref[a:b] >= 0, M_local + rank[pref[a:b].clamp(min=0)],
                                                        -1 - pref[a:b]), g_tgt, g_delay, g_w, n)
    del g_tgt, g_delay, g_w
    net.prepare()
    assert net.count("r_val") == used_idx.numel()
    R = net.tensor("r_val").long()
    r_off = torch.from_numpy(net.array("r_off").astype(np.int64)).cuda()
    sigma_of = torch.searchsorted(r_off[1:], torch.arange(R.numel(), device="cuda"), right=True)
    a_of, s_of = sigma_of // P, sigma_of % P
    got_pref = a_of * G + torch.from_numpy(base[:-1]).cuda()[s_of] + R
    assert torch.equal(got_pref, used_idx), "image map differs from the used remote sources"
    src, tgt, rp = net.tensor("src"), net.tensor("tgt"), net.tensor("row_ptr")
    _check_sorted_and_csr(torch, src, tgt, rp, n)
    after = _hash_sums(torch, lambda a, b: src[a:b], tgt, net.tensor("delay"), net.tensor("weight"), n)
    assert before == after, "sorted network is not the generated multiset under the image numbering"
    # collective I: image index where the passed source has an image, else -1
    H, I = net.tensor("h_val").long(), net.tensor("i_val").long()
    h_off = net.array("h_off").astype(np.int64)
    for sigma in (1, 511, P - 1):
        h = H[h_off[sigma]:h_off[sigma + 1]]
        i = I[h_off[sigma]:h_off[sigma + 1]]
        p = 1 * G + int(base[sigma]) + h
        has = used[p].bool()
        assert torch.equal(i >= 0, has)
        assert torch.equal(i[has], M_local + rank[p[has]])
    log(f"collective full: {n} connections, {R.numel()} images")
    net.close()


def test_multiarea_p2p_full_size():
    torch = _torch()
    script = W.multiarea_p2p()
    net0 = _build(script, 0)
    ref = oracle.run_script(script, 0, declare_only=True)
    k = _sample_generation(net0, ref, n_samples=300)
    log(f"multiarea full: {k} sampled elements equal the oracle")
    net0.prepare()
    s_off = net0.array("s_off").astype(np.int64)
    S = net0.tensor("s_val")
    src, tgt, rp = net0.tensor("src"), net0.tensor("tgt"), net0.tensor("row_ptr")
    _check_sorted_and_csr(torch, src, tgt, rp, net0.count("src"))
    net0.close()
    for tau in (1, 31):
        net = _build(script, tau)
        net.prepare()
        r_off = net.array("r_off").astype(np.int64)
        R = net.tensor("r_val")
        assert torch.equal(S[s_off[tau]:s_off[tau + 1]], R[r_off[0]:r_off[1]]), f"S on 0 != R on {tau}"
        net.close()


def _served_build(script, budget, batched):
    reqs = [op for op in script["ops"] if op[0] == "connect"]
    net = snnc.Network(1, 0, script["seed"], script["dt"])
    net.set_resident_budget(budget)
    net.reserve(budget // 14)
    for op in script["ops"]:
        if op[0] == "create":
            net.create(op[1], op[2])
    admitted = []
    for k, op in enumerate(reqs):
        _, src, tgt, conn, syn, alpha = op
        try:
            (net.submit if batched else net.connect)(src, tgt, conn, syn, alpha)
            admitted.append(k)
        except snnc.SnncError as e:
            assert e.code == -3, e
        if batched and admitted and len(admitted) % 256 == 0:
            net.flush()
    if batched:
        net.flush()
    net.sync()
    return net, admitted


def test_served_full_size():
    """10,000 uneven requests against a 64 GiB resident budget, built in fused
    batches as the bench builds them: the admitted requests and their
    connection counts equal the per-call build's; sampled connections of the
    rules whose elements are independent equal the oracle's replay of their
    element (element = position for fixed in/out-degree and total number
    with multapses and autapses, the source ordinal for one-to-one, the pair
    index for Bernoulli); calls of up to 20,000 connections of every rule
    (Floyd's sampling, first-N-valid candidates) equal the oracle's generation
    of the whole call."""
    _torch()
    script = W.served_requests()
    budget = 64 << 30
    reqs = [op for op in script["ops"] if op[0] == "connect"]
    net, adm = _served_build(script, budget, batched=True)
    off = net.array("call_off").astype(np.int64)
    per_call, adm_p = _served_build(script, budget, batched=False)
    off_p = per_call.array("call_off").astype(np.int64)
    per_call.close()
    assert adm == adm_p
    np.testing.assert_array_equal(off, off_p)
    log(f"served full: {len(adm)} admitted, {off[-1]} connections")
    kept = dict(script)
    kept["ops"] = [op for op in script["ops"] if op[0] == "create"] + [reqs[k] for k in adm]
    ref = oracle.run_script(kept, 0, declare_only=True)
    rng = np.random.default_rng(3)
    n_elem = n_full = 0
    for c, k in enumerate(adm):
        _, src, tgt, conn, syn, alpha = reqs[k]
        a, b = int(off[c]), int(off[c + 1])
        if b == a:
            continue
        rule = conn["rule"]
        aut, mult = conn.get("autapses", True), conn.get("multapses", True)
        independent = (rule in ("fixed_indegree", "fixed_outdegree") and mult) or \
                      (rule == "fixed_total_number" and mult and aut) or rule in ("one_to_one", "pairwise_bernoulli")
        if independent and c % 3 == 0:
            for p in np.unique(rng.integers(a, b, size=4)):
                p = int(p)
                got = {n: net.array_range("gen_" + n, p, 1)[0] for n in ("src", "tgt", "delay", "weight")}
                if rule == "one_to_one":
                    e = int(got["src"])
                elif rule == "pairwise_bernoulli":
                    n_s = sum(s[2] for s in src)
                    e = (int(got["tgt"]) - tgt[0][1]) * n_s + int(got["src"])
                else:
                    e = p - a
                r = ref.element(c, e)
                assert r is not None, (c, rule, e)
                assert (got["src"], got["tgt"], got["delay"]) == (r["src"], r["tgt"], r["delay"]), (c, rule, p)
                assert ulp_diff(np.array([got["weight"]], np.float32), np.array([r["weight"]], np.float32)) <= 2
                n_elem += 1
        if b - a <= 20000 and (not independent or c % 7 == 0):
            want = ref.call_range(c, 0, 0, 2**63, b - a + 1)
            assert want["src"].size == b - a, (c, rule, want["src"].size, b - a)
            np.testing.assert_array_equal(net.array_range("gen_src", a, b - a), want["src"])
            np.testing.assert_array_equal(net.array_range("gen_tgt", a, b - a), want["tgt"])
            np.testing.assert_array_equal(net.array_range("gen_delay", a, b - a), want["delay"])
            assert ulp_diff(net.array_range("gen_weight", a, b - a), want["weight"]) <= 2
            n_full += 1
    log(f"served full: {n_elem} sampled elements, {n_full} whole calls equal the oracle")
    net.close()
