"""GPU checks of served (batched) construction: a stream of uneven requests
admitted against a resident budget gives bit-identical networks whether it
is built per call or in fused batches, and both equal the oracle's build of
the admitted requests."""
import numpy as np
import pytest

import oracle
import paper_2512_09502_amd as snnc
from fullsize_oracle import served_admission
from gpu_util import GEN_ARRAYS, PREP_ARRAYS, compare, log
from paper_2512_09502_amd import workloads as W

pytestmark = pytest.mark.gpu


def _served_script(n=120, size_max=3e4, seed=7):
    return W.served_requests(n_requests=n, n_pops=12, pop_min=200, pop_max=3000, size_min=10, size_max=size_max,
                             seed=seed)


def _build(script, mode, budget, batch=17, fuse=True, reserve=0):
    import torch
    torch.cuda.set_device(0)
    net = snnc.Network(1, 0, script["seed"], script["dt"])
    net.tune("fuse_batches", int(fuse))
    if budget:
        net.set_resident_budget(budget)
    if reserve:
        net.reserve(reserve)
    rejected, submitted = [], 0
    if mode.startswith("many"):   # "many<chunk>": snnc_submit_many over chunks of the request stream
        chunk = int(mode[4:])
        pending = []

        def submit_chunk():
            res = net.submit_many([req for _, req in pending])
            for (k, _), (status, cid) in zip(pending, res):
                if status != 0:
                    rejected.append((k, status))
                    assert cid is None
            pending.clear()
            net.flush()
        for k, op in enumerate(script["ops"]):
            if op[0] == "create":
                net.create(op[1], op[2])
                continue
            pending.append((k, op[1:]))
            if len(pending) == chunk:
                submit_chunk()
        submit_chunk()
        net.sync()
        gen = {k: net.array(k) for k in GEN_ARRAYS}
        net.prepare()
        out = {k: net.array(k) for k in PREP_ARRAYS}
        out.update(gen)
        net.close()
        return out, rejected
    for k, op in enumerate(script["ops"]):
        if op[0] == "create":
            net.create(op[1], op[2])
            continue
        _, src, tgt, conn, syn, alpha = op
        fn = net.connect if mode == "per_call" else net.submit
        try:
            fn(src, tgt, conn, syn, alpha)
            submitted += 1
        except snnc.SnncError as e:
            rejected.append((k, e.code))
            continue
        if mode == "batched" and submitted % batch == 0:
            net.flush()
    if mode == "batched":
        net.flush()
    gen = {k: net.array(k) for k in GEN_ARRAYS} if mode != "batched" else None
    net.sync()
    if mode == "batched":
        gen = {k: net.array(k) for k in GEN_ARRAYS}
    net.prepare()
    out = {k: net.array(k) for k in PREP_ARRAYS}
    out.update(gen)
    net.close()
    return out, rejected


@pytest.mark.parametrize("fuse", [True, False])
def test_batched_equals_per_call_under_budget(fuse):
    script = _served_script()
    total = sum(int(op[3].get("n", 0)) for op in script["ops"] if op[0] == "connect")
    budget = 14 * 200000 + 50000      # rejects part of the stream
    a, rej_a = _build(script, "per_call", budget)
    b, rej_b = _build(script, "batched", budget, fuse=fuse)
    log(f"served: {len(rej_a)} rejected of {len(script['ops'])} ops, {a['src'].size} connections")
    assert rej_a == rej_b
    assert any(code == -3 for _, code in rej_a), "the budget should reject some requests"
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    # the oracle's own admission (its counts under the documented resident
    # cost) rejects the same requests; its build of the admitted ones is the network
    status, admitted, _ = served_admission(script, budget, workers=2)
    conn_at = [k for k, op in enumerate(script["ops"]) if op[0] == "connect"]
    assert [(conn_at[i], st) for i, st in enumerate(status) if st != 0] == rej_a
    kept = dict(script)
    keep = {conn_at[i] for i in admitted}
    kept["ops"] = [op for k, op in enumerate(script["ops"]) if op[0] == "create" or k in keep]
    ref = oracle.run_script(kept, 0)
    for k in GEN_ARRAYS + PREP_ARRAYS:
        compare(k, b[k], ref.array(k), "served")


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_submit_many_streams_equal_oracle(seed):
    """Streams with requests up to 3e5 connections (candidate windows on the
    filtered and the one-workgroup first-occurrence paths, Bernoulli counts
    over several hundred tiles, Floyd degrees in every workgroup shape),
    submitted in chunks of 64: admission equals the oracle's and the network
    equals the oracle's build of the admitted requests."""
    script = _served_script(n=150, size_max=3e5, seed=seed)
    budget = 14 * 3_000_000
    b, rej_b = _build(script, "many64", budget)
    status, admitted, _ = served_admission(script, budget, workers=2)
    conn_at = [k for k, op in enumerate(script["ops"]) if op[0] == "connect"]
    assert [(conn_at[i], st) for i, st in enumerate(status) if st != 0] == rej_b
    kept = dict(script)
    keep = {conn_at[i] for i in admitted}
    kept["ops"] = [op for k, op in enumerate(script["ops"]) if op[0] == "create" or k in keep]
    ref = oracle.run_script(kept, 0)
    log(f"served seed {seed}: {len(admitted)} admitted, {b['src'].size} connections, {len(rej_b)} rejected")
    for k in GEN_ARRAYS + PREP_ARRAYS:
        compare(k, b[k], ref.array(k), f"served seed {seed}")


@pytest.mark.parametrize("chunk", [1, 13, 200])
def test_submit_many_equals_submit(chunk):
    """Batched submission (one device wait per chunk for the counts) admits
    the same requests, assigns the same call ids and builds the same network
    as one submit per request, with requests rejected by the budget and
    invalid ones inside the chunks (so later requests' assumed ids move)."""
    script = _served_script(n=160, seed=11)
    # two invalid requests: a receptor port, and a degree above the candidates without multapses
    ops = script["ops"]
    firsts = [k for k, op in enumerate(ops) if op[0] == "connect"]
    bad = dict(ops[firsts[5]][4]); bad["port"] = 1
    ops.insert(firsts[5] + 1, ("connect", ops[firsts[5]][1], ops[firsts[5]][2], ops[firsts[5]][3], bad, -1))
    src = ops[firsts[9]][1]
    ops.insert(firsts[9] + 1, ("connect", src, src, {"rule": "fixed_indegree", "n": 10**6, "multapses": False},
                               ops[firsts[9]][4], -1))
    budget = 14 * 200000 + 50000
    a, rej_a = _build(script, "batched", budget)
    b, rej_b = _build(script, f"many{chunk}", budget)
    log(f"submit_many chunk {chunk}: {len(rej_a)} rejected, {a['src'].size} connections")
    assert rej_a == rej_b
    assert any(code == -3 for _, code in rej_a) and any(code == -1 for _, code in rej_a)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_submit_many_edges():
    """An empty list, a list of only invalid requests, a request past the
    budget between admitted ones, and the state check after prepare."""
    import torch
    torch.cuda.set_device(0)
    net = snnc.Network(1, 0, 3, 0.1)
    a = net.create(0, 1000)
    syn = {"weight": {"kind": "const", "mean": 0.5}, "delay": {"kind": "const", "mean": 1.0}}
    assert net.submit_many([]) == []
    bad = ([a], [a], {"rule": "one_to_one"}, dict(syn, port=2))
    assert net.submit_many([bad, bad]) == [(-1, None), (-1, None)]
    net.set_resident_budget(14 * 60000 + 4096)
    small = ([a], [a], {"rule": "pairwise_bernoulli", "p": 0.02}, syn)
    big = ([a], [a], {"rule": "fixed_total_number", "n": 100000, "autapses": False}, syn)
    res = net.submit_many([small, big, small])
    assert [st for st, _ in res] == [0, -3, 0] and [cid for _, cid in res] == [0, None, 1]
    net.flush()
    net.prepare()
    n = net.count("src")
    assert 30000 < n < 50000, n
    with pytest.raises(snnc.SnncError) as e:
        net.submit_many([small])
    assert e.value.code == -4
    net.close()


def test_counting_lane_with_large_requests():
    """Admission counts run on their own stream while earlier batches generate;
    requests up to 1e6 connections make the counting lane reuse its large
    blocks (sort buffers of total number without multapses, tile counts)
    while generation that reads their predecessors may still be queued.  The
    build equals the one-stream build (per call, no budget), which the other
    parity tests check against the oracle."""
    script = W.served_requests(n_requests=150, n_pops=12, pop_min=2000, pop_max=50000, size_min=1e3, size_max=1e6,
                               seed=11)
    a, rej_a = _build(script, "per_call", 0)
    b, rej_b = _build(script, "batched", 1 << 40, batch=7, reserve=30_000_000)
    c, rej_c = _build(script, "per_call", 1 << 40)
    log(f"counting lane: {a['src'].size} connections")
    assert rej_a == rej_b == rej_c == []
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
        np.testing.assert_array_equal(a[k], c[k], err_msg=k)


def test_served_poll_and_flush_order():
    import torch
    torch.cuda.set_device(0)
    script = _served_script(n=40, seed=9)
    net = snnc.Network(1, 0, script["seed"], script["dt"])
    ids = []
    for op in script["ops"]:
        if op[0] == "create":
            net.create(op[1], op[2])
        else:
            _, src, tgt, conn, syn, alpha = op
            try:
                ids.append(net.submit(src, tgt, conn, syn, alpha))
            except snnc.SnncError:
                pass
    assert not any(net.poll(i) for i in ids[:3])      # nothing flushed yet
    net.flush()
    net.sync()
    assert all(net.poll(i) for i in ids)
    net.prepare()
    with pytest.raises(snnc.SnncError):
        net.flush()
    net.close()


@pytest.mark.parametrize("reserve", [0, 40_000_000])
def test_generation_blocks_equal_doubling(reserve):
    """Generation arrays in mapped fixed-size blocks (grown as calls and
    admitted requests need them; 2^26 connections per block, so these
    8.2e7-connection builds cross block boundaries inside calls) equal the
    doubling arrays, before and after Prepare, per call and in batches."""
    import torch
    torch.cuda.set_device(0)
    b = W._Builder(1, seed=3)
    a = b.create(0, 60000)
    c = b.create(0, 50000)
    syn = {"weight": {"kind": "normal", "mean": 0.1, "sd": 0.01},
           "delay": {"kind": "normal", "mean": 1.5, "sd": 0.75, "lo": 0.1}}
    b.connect([a], [c], {"rule": "fixed_indegree", "n": 700}, syn)
    b.connect([c], [a], {"rule": "fixed_outdegree", "n": 520}, syn)
    b.connect([a], [a], {"rule": "fixed_total_number", "n": 21_000_000, "autapses": False}, syn)
    script = b.script("blocks")
    out = []
    for blocks, batched in ((0, False), (1, False), (1, True)):
        net = snnc.Network(1, 0, script["seed"], script["dt"])
        try:
            net.tune("gen_blocks", blocks)
        except snnc.SnncError as e:
            pytest.skip(f"no virtual memory management: {e}")
        if reserve:
            net.reserve(reserve)
        if batched:
            net.set_resident_budget(1 << 40)
        for op in script["ops"]:
            if op[0] == "create":
                net.create(op[1], op[2])
        ops = [op[1:] for op in script["ops"] if op[0] == "connect"]
        if batched:
            assert [st for st, _ in net.submit_many(ops)] == [0, 0, 0]
            net.flush()
        else:
            for op in ops:
                net.connect(*op)
        net.sync()
        n = net.count("gen_src")
        assert n == 50000 * 700 + 50000 * 520 + 21_000_000
        got = {k: net.array_range(k, 0, n)[::997].copy() for k in GEN_ARRAYS}
        net.prepare()
        got.update({k: net.array(k) for k in ("src", "tgt", "delay", "weight", "row_ptr")})
        net.close()
        out.append(got)
    for got in out[1:]:
        for k in out[0]:
            np.testing.assert_array_equal(out[0][k], got[k], err_msg=k)
    log(f"generation blocks (reserve {reserve}): equal to the doubling arrays")


def test_fused_grid_autotuner():
    """The fused-launch autotuner picks one of its grids, caches it for the
    device (a second call returns at once, new contexts take it), and the
    grid changes nothing in the network."""
    import torch
    torch.cuda.set_device(0)
    net = snnc.Network(1, 0, 1, 0.1)
    r = net.autotune_fused(3_000_000)
    assert r["fused_wgs_per_cu"] in (1, 2, 4, 8, 16, 32)
    again = net.autotune_fused(3_000_000)
    assert again["fused_wgs_per_cu"] == r["fused_wgs_per_cu"] and again["ms"] == -1.0
    net.close()
    script = _served_script(n=60, seed=21)
    a, _ = _build(script, "batched", 1 << 40)                     # the tuned grid (taken at init)
    outs = []
    for w in (1, 32):
        net = snnc.Network(1, 0, script["seed"], script["dt"])
        net.tune("fused_wgs_per_cu", w)
        net.set_resident_budget(1 << 40)
        for op in script["ops"]:
            if op[0] == "create":
                net.create(op[1], op[2])
        for k0 in range(0, 60, 17):
            net.submit_many([op[1:] for op in script["ops"] if op[0] == "connect"][k0:k0 + 17])
            net.flush()
        net.prepare()
        outs.append({k: net.array(k) for k in PREP_ARRAYS})
        net.close()
    for o in outs:
        for k in PREP_ARRAYS:
            np.testing.assert_array_equal(a[k], o[k], err_msg=k)
