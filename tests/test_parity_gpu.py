"""GPU parity: the HIP library against the oracle on the same seeded scripts,
every output array element by element (integers bit-exact, weights within
2 fp32 ulp), at sizes that span many tiles and ragged tails."""
import numpy as np
import pytest

import oracle
from gpu_util import compare, compare_all, log
from paper_2512_09502_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


def test_philox_blocks_match_oracle():
    import paper_2512_09502_amd as snnc
    net = snnc.Network(1, 0, 1, 0.1)
    rng = np.random.default_rng(1)
    for seed, call, e0, purpose in [(1, 0, 0, 0), (0xFFFFFFFF, 7, 2**32 - 3, 1), (12345, 99, 2**40 + 17, 2)]:
        got = net.philox_blocks(seed, call, e0, purpose, 300)
        for i in rng.integers(0, 300, size=40):
            e = e0 + int(i)
            ref = oracle.philox([e & 0xFFFFFFFF, e >> 32, purpose, 0], [seed, call])
            assert got[i].tolist() == ref.tolist()
    net.close()


def test_balanced_small_full():
    n = compare_all(W.balanced_small(), 0)
    assert n == 100000


@pytest.mark.parametrize("scale", [0.02, 0.05])
def test_column8_scaled(scale):
    s = W.column8(scale=scale)
    n = compare_all(s, 0)
    log(f"column8 scale={scale}: {n} connections")


def test_multiarea_p2p_scaled():
    s = W.multiarea_p2p(P=6, n_e=800, n_i=200, k_e=40, k_i=10, k_remote_max=12)
    for pl in (0, 3):
        compare_all(s, pl)


@pytest.mark.parametrize("variant", range(12))
def test_number_variants(variant):
    """Every tile shape of the image-numbering pass (block size, items per
    thread, payload loaded before or after the look-back) gives the oracle's
    arrays, on networks with remote sources over many tiles."""
    for s in (W.multiarea_p2p(P=6, n_e=2000, n_i=500, k_e=40, k_i=10, k_remote_max=12),
              W.balanced_collective(P=12, n_e=400, n_i=100, k_e=90, k_i=22)):
        s["tune"] = {"number_variant": variant}
        compare_all(s, 1)


def test_balanced_collective_scaled():
    s = W.balanced_collective(P=12, n_e=400, n_i=100, k_e=90, k_i=22)
    for pl in (0, 11):
        compare_all(s, pl)


@pytest.mark.parametrize("aut,mult", [(True, True), (False, True), (True, False), (False, False)])
def test_total_number_over_several_hosts(aut, mult):
    """Fixed total number with targets on four hosts: every host keeps its
    part of the first N valid candidates."""
    b = W._Builder(4, seed=99)
    pops = [b.create(h, 300 + 50 * h) for h in range(4)]
    b.connect(pops, pops[1:], {"rule": "fixed_total_number", "n": 60000, "autapses": aut, "multapses": mult},
              SYN_N, -1)
    b.connect([pops[2]], pops, {"rule": "fixed_total_number", "n": 9000, "autapses": aut, "multapses": mult},
              SYN_N, 0)
    s = b.script(f"total_dist_{int(aut)}{int(mult)}")
    for pl in range(4):
        n = compare_all(s, pl)
        log(f"total number over hosts, P_local={pl}: {n} connections")


@pytest.mark.parametrize("in_scale", [1, 4, 10])
def test_balanced_indegree_scaled(in_scale):
    """In-degree sweep at a fixed connection count (fewer sources, larger K)."""
    s = W.balanced_indegree(in_scale, P=6, n_e=400, n_i=100, k_e=30, k_i=8)
    for pl in (0, 5):
        n = compare_all(s, pl)
        log(f"indegree x{in_scale} P_local={pl}: {n} connections")


@pytest.mark.parametrize("seed", range(16))
def test_random_tiny(seed):
    s = W.random_tiny(seed)
    for pl in range(s["P"]):
        compare_all(s, pl)


SYN_N = {"weight": {"kind": "normal", "mean": 0.3, "sd": 0.2},
         "delay": {"kind": "normal", "mean": 2.0, "sd": 1.0, "lo": 0.2}}


def _one(rule_conn, n_src=3000, n_tgt=2500, P=1, src_host=0, tgt_host=0, alpha=-1):
    b = W._Builder(P, seed=77)
    pops = {}
    for h in range(P):
        pops[h] = b.create(h, max(n_src, n_tgt))
    src = [(src_host, 0, n_src)]
    tgt = [(tgt_host, 100, n_tgt - 100)] if n_tgt > 100 else [(tgt_host, 0, n_tgt)]
    b.connect(src, tgt, rule_conn, SYN_N, alpha)
    return b.script("one_" + rule_conn["rule"])


@pytest.mark.parametrize("conn", [
    {"rule": "fixed_indegree", "n": 37, "autapses": False, "multapses": False},
    {"rule": "fixed_indegree", "n": 1, "autapses": False, "multapses": False},
    {"rule": "fixed_indegree", "n": 32, "autapses": True, "multapses": False},
    {"rule": "fixed_indegree", "n": 33, "autapses": False, "multapses": False},
    {"rule": "fixed_outdegree", "n": 7, "autapses": True, "multapses": False},
    {"rule": "fixed_outdegree", "n": 32, "autapses": False, "multapses": False},
    {"rule": "fixed_indegree", "n": 300, "autapses": True, "multapses": False},
    {"rule": "fixed_outdegree", "n": 41, "autapses": False, "multapses": True},
    {"rule": "fixed_outdegree", "n": 23, "autapses": False, "multapses": False},
    {"rule": "fixed_total_number", "n": 200000, "autapses": False, "multapses": True},
    {"rule": "fixed_total_number", "n": 150000, "autapses": True, "multapses": False},
    {"rule": "fixed_total_number", "n": 120000, "autapses": False, "multapses": False},
    {"rule": "fixed_total_number", "n": 1100000, "autapses": True, "multapses": False},   # window above 2^20: sort path
    {"rule": "pairwise_bernoulli", "p": 0.013, "autapses": False},
    {"rule": "pairwise_bernoulli", "p": 1.0, "autapses": True},
    {"rule": "one_to_one", "autapses": False},
])
def test_rules_with_flags(conn):
    if conn["rule"] == "one_to_one":
        s = _one(conn, n_src=2400, n_tgt=2500)
    elif conn["rule"] == "pairwise_bernoulli":
        s = _one(conn, n_src=900, n_tgt=700)
    else:
        s = _one(conn)
    compare_all(s, 0)


@pytest.mark.parametrize("rule,k,n_src,n_tgt,aut", [
    ("fixed_indegree", 2990, 3000, 400, False),    # K close to the candidate count: long fallback chains
    ("fixed_indegree", 8192, 9000, 300, False),    # largest degree of the workgroup sampler
    ("fixed_indegree", 64, 64, 400, False),        # K = all candidates
    ("fixed_outdegree", 8000, 200, 8300, False),
    ("fixed_outdegree", 33, 500, 133, True),       # K = all targets
])
def test_large_degree_without_multapses(rule, k, n_src, n_tgt, aut):
    conn = {"rule": rule, "n": k, "autapses": aut, "multapses": False}
    compare_all(_one(conn, n_src=n_src, n_tgt=n_tgt), 0)


@pytest.mark.parametrize("rule", ["fixed_outdegree", "pairwise_bernoulli", "fixed_indegree", "one_to_one"])
def test_remote_rules_all_hosts(rule):
    # sources on host 1, targets spread over hosts 0..2: every host's share,
    # including the regenerated point-to-point lists on host 1
    b = W._Builder(3, seed=5)
    p = [b.create(h, 500) for h in range(3)]
    conn = {"rule": rule, "n": 9, "p": 0.05, "autapses": True, "multapses": rule != "fixed_outdegree"}
    tgt = [(0, 0, 500), (2, 0, 500), (1, 0, 500)]
    src = [(1, 0, 500)] if rule != "one_to_one" else [(1, 0, 500), (0, 0, 500), (2, 0, 500)]
    b.connect(src, tgt, conn, SYN_N, -1)
    b.connect(src, tgt, conn, SYN_N, 0)
    s = b.script("remote_" + rule)
    for pl in range(3):
        compare_all(s, pl)


@pytest.mark.parametrize("in_lds", [1, 0])
def test_mark_rows(in_lds):
    # point-to-point regeneration on the source host, with the bit rows marked
    # in LDS (one OR per word and workgroup) or with a global atomic per draw
    b = W._Builder(3, seed=9)
    src = b.create(0, 20000)
    tgt = b.create(1, 3000)
    other = b.create(2, 500)
    for rule in ("fixed_indegree", "fixed_outdegree", "fixed_total_number"):
        n = {"fixed_indegree": 40, "fixed_outdegree": 7, "fixed_total_number": 150000}[rule]
        conn = {"rule": rule, "n": n, "autapses": True, "multapses": True}
        b.connect([src], [tgt] if rule != "fixed_outdegree" else [tgt, other], conn, SYN_N, -1)
    s = b.script(f"mark_rows_{in_lds}")
    s["tune"] = {"mark_in_lds": in_lds}
    for pl in (0, 1, 2):
        compare_all(s, pl)


def test_mark_row_of_the_largest_lds_size():
    # a bit row of 2^19 neurons fills the 64 KB of LDS the marking kernel may
    # use: its send lists equal those of the global-atomic path (which the
    # oracle pins at smaller sizes)
    import paper_2512_09502_amd as snnc
    b = W._Builder(2, seed=13)
    src = b.create(0, 1 << 19)
    tgt = b.create(1, 2000)
    b.connect([src], [tgt], {"rule": "fixed_indegree", "n": 30, "autapses": True, "multapses": True}, SYN_N, -1)
    s = b.script("mark_row_max")
    out = []
    for in_lds in (1, 0):
        s["tune"] = {"mark_in_lds": in_lds}
        net = snnc.run_script(s, 0)
        out.append({k: net.array(k) for k in ("s_off", "s_val", "tp_ptr", "t_val", "p_val")})
        net.close()
    for k in out[0]:
        np.testing.assert_array_equal(out[0][k], out[1][k], err_msg=k)
    assert out[0]["s_val"].size > 50000


@pytest.mark.parametrize("k", [9, 50])
def test_remote_outdegree_without_multapses(k):
    # counting, writing and point-to-point marking through both samplers (small and large K)
    b = W._Builder(3, seed=8)
    p = [b.create(h, 400) for h in range(3)]
    conn = {"rule": "fixed_outdegree", "n": k, "autapses": False, "multapses": False}
    b.connect([(1, 0, 400), (2, 0, 100)], [(0, 0, 400), (2, 0, 400), (1, 0, 400)], conn, SYN_N, -1)
    s = b.script(f"remote_outdegree_k{k}")
    for pl in range(3):
        compare_all(s, pl)


def test_edge_cases():
    b = W._Builder(2, seed=3)
    a = b.create(0, 1)
    c = b.create(1, 5)
    d0 = {"kind": "const", "mean": 0.1}
    syn = {"weight": {"kind": "const", "mean": 1.0}, "delay": d0}
    b.connect([a], [a], {"rule": "fixed_indegree", "n": 0}, syn)                    # K = 0
    b.connect([a], [a], {"rule": "pairwise_bernoulli", "p": 0.0}, syn)              # p = 0
    b.connect([a], [a], {"rule": "fixed_indegree", "n": 3}, syn)                    # single neuron, autapses
    b.connect([c], [a], {"rule": "fixed_total_number", "n": 7}, syn, 0)             # remote sources, group 0
    b.connect([a, c], [a], {"rule": "one_to_one", "autapses": False}, syn)          # invalid: sizes differ
    s = b.script("edge")
    for pl in range(2):
        compare_all(s, pl)
    # no connection at all
    b = W._Builder(1)
    b.create(0, 10)
    compare_all(b.script("empty"), 0)


@pytest.mark.parametrize("wave_max", [0, 1024, 8192])
@pytest.mark.parametrize("rule,k,n_src,n_tgt,aut", [
    ("fixed_indegree", 37, 500, 300, False),
    ("fixed_indegree", 100, 400, 300, True),
    ("fixed_indegree", 200, 600, 200, False),
    ("fixed_indegree", 1000, 1200, 200, True),
    ("fixed_indegree", 2990, 3000, 100, False),
    ("fixed_outdegree", 300, 100, 900, False),
    ("fixed_outdegree", 1500, 50, 2000, True),
])
def test_floyd_workgroup_shapes(rule, k, n_src, n_tgt, aut, wave_max):
    # one-wave, 256- and 1024-thread workgroups of the parallel Floyd sampler give the oracle's
    # sets: padded degrees of 1 to 16 keys per thread sorted in registers, the rest in LDS
    conn = {"rule": rule, "n": k, "autapses": aut, "multapses": False}
    s = _one(conn, n_src=n_src, n_tgt=n_tgt)
    s["tune"] = {"floyd_wave_max": wave_max}
    compare_all(s, 0)


@pytest.mark.parametrize("wave_max", [0, 8192])
@pytest.mark.parametrize("rule,k,n_src,n_tgt,aut", [
    ("fixed_indegree", 5000, 524_287, 8, False),        # (value << 13 | step) just fits 32 bits
    ("fixed_indegree", 5000, 524_288, 8, True),         # one more candidate: 64-bit keys
    ("fixed_indegree", 2100, 1_048_577, 6, False),      # padded degree 4096, 64-bit keys
    ("fixed_outdegree", 4100, 6, 524_388, False),       # 524,288 targets: 64-bit keys
])
def test_floyd_sort_key_widths(rule, k, n_src, n_tgt, aut, wave_max):
    # the workgroup sampler sorts 32-bit keys while the candidate set times the padded degree
    # stays below 2^32, 64-bit keys beyond; both widths give the oracle's sets
    conn = {"rule": rule, "n": k, "autapses": aut, "multapses": False}
    s = _one(conn, n_src=n_src, n_tgt=n_tgt)
    s["tune"] = {"floyd_wave_max": wave_max}
    compare_all(s, 0)


@pytest.mark.parametrize("aut", [False, True])
@pytest.mark.parametrize("p", [1.0, 0.5])
@pytest.mark.parametrize("n_src,n_tgt", [(1, 1), (2, 7), (3, 50), (5, 90), (7, 33), (1030, 300)])
def test_bernoulli_block_edges(n_src, n_tgt, p, aut):
    # source counts that leave a target's pairs starting and ending inside Philox blocks, with the
    # targets among the sources so that the excluded autapse falls at every position of a block
    conn = {"rule": "pairwise_bernoulli", "p": p, "autapses": aut}
    compare_all(_one(conn, n_src=n_src, n_tgt=n_tgt), 0)


@pytest.mark.parametrize("tune", [{"total_hash_max": 0}, {"total_small_max": 0}, {"total_small_max": 1 << 15}],
                         ids=["sorted", "filtered", "one_workgroup"])
@pytest.mark.parametrize("n,aut,n_src,n_tgt", [(1_100_000, True, 3000, 2500), (150_000, False, 3000, 2500),
                                               (5_000_000, False, 3000, 2500), (990, False, 20, 150),
                                               (40_000, True, 200, 300), (5_000, False, 3000, 2500),
                                               (20_000, True, 3000, 2500), (1, False, 3000, 2500)])
def test_total_number_first_occurrence_paths(n, aut, n_src, n_tgt, tune):
    # first candidates of each pair by sorting the pair keys, by filtered hashing in separate launches,
    # and (windows up to 2^15 candidates) in one workgroup; the dense cases (most candidates repeat a
    # pair) send most candidates through the exact table
    conn = {"rule": "fixed_total_number", "n": n, "autapses": aut, "multapses": False}
    s = _one(conn, n_src=n_src, n_tgt=n_tgt)
    s["tune"] = dict(tune)
    compare_all(s, 0)


def _many_segments_script(conn):
    # node sets of five and six segments from eight populations, sources and targets overlapping:
    # the calls' run tables are longer than what travels inline with the kernel arguments
    b = W._Builder(1, seed=91)
    pops = [b.create(0, n) for n in (700, 300, 500, 900, 200, 600, 400, 800)]

    def seg(p, a, n):
        return (0, pops[p][1] + a, n)
    tgt = [seg(0, 200, 400), seg(1, 0, 300), seg(3, 450, 400), seg(4, 0, 200), seg(5, 0, 600), seg(6, 50, 300)]
    if conn["rule"] == "one_to_one":   # same size as the targets, shifted
        src = [seg(0, 150, 400), seg(1, 0, 300), seg(3, 400, 400), seg(4, 0, 200), seg(5, 0, 600), seg(7, 0, 300)]
    else:
        src = [seg(0, 0, 500), seg(2, 100, 300), seg(3, 0, 900), seg(5, 200, 300), seg(7, 0, 600)]
    b.connect(src, tgt, conn, SYN_N)
    b.connect(tgt, src, conn, SYN_N)
    return b.script("many_segments_" + conn["rule"])


MANY_SEGMENT_RULES = [
    {"rule": "fixed_indegree", "n": 40, "autapses": False, "multapses": False},
    {"rule": "fixed_indegree", "n": 9, "autapses": False, "multapses": True},
    {"rule": "fixed_outdegree", "n": 12, "autapses": False, "multapses": False},
    {"rule": "fixed_outdegree", "n": 7, "autapses": True, "multapses": True},
    {"rule": "pairwise_bernoulli", "p": 0.05, "autapses": False, "multapses": True},
    {"rule": "one_to_one", "autapses": False, "multapses": True},
    {"rule": "fixed_total_number", "n": 30000, "autapses": False, "multapses": False},
    {"rule": "fixed_total_number", "n": 20000, "autapses": True, "multapses": True},
]


@pytest.mark.parametrize("conn", MANY_SEGMENT_RULES, ids=lambda c: f"{c['rule']}-{c.get('n', c.get('p'))}")
def test_many_segment_sets(conn):
    # per call: the run tables go to the device (more runs than travel inline)
    compare_all(_many_segments_script(conn), 0)


@pytest.mark.parametrize("conn", MANY_SEGMENT_RULES, ids=lambda c: f"{c['rule']}-{c.get('n', c.get('p'))}")
def test_many_segment_sets_batched(conn):
    # the same calls submitted as one batch: fused descriptors whose run tables are patched to the
    # batch's one device copy, and Floyd calls that keep their own synapse-value pass
    import paper_2512_09502_amd as snnc
    s = _many_segments_script(conn)
    net = snnc.Network(1, 0, s["seed"], s["dt"])
    reqs = []
    for op in s["ops"]:
        if op[0] == "create":
            net.create(op[1], op[2])
        else:
            reqs.append(op[1:])
    assert all(status == 0 for status, _ in net.submit_many(reqs))
    net.flush()
    net.prepare()
    ref = oracle.run_script(s, 0)
    for k in ("src", "tgt", "delay", "weight", "row_ptr"):
        compare(k, net.array(k), ref.array(k), s["name"] + " batched")
    net.close()


@pytest.mark.parametrize("p", [1e-4, 2e-6])
def test_bernoulli_sparse_tiles(p):
    # most tiles of 4,096 pairs hold no connection (the writing pass skips them) or a single one
    conn = {"rule": "pairwise_bernoulli", "p": p, "autapses": False}
    compare_all(_one(conn, n_src=3000, n_tgt=2500), 0)


def _batch_mix_script():
    # Floyd calls (no multapses) of degrees on both sides of the small sampler's limit of 32 and
    # Bernoulli calls of sizes that end inside a tile, single-segment sets (run tables inline),
    # among fusable calls: a batch's fused launch then holds small-sampler units, whole Bernoulli
    # writing tiles (after alignment padding) and connection items of other calls
    b = W._Builder(1, seed=57)
    a = b.create(0, 900)
    c = b.create(0, 700)
    d = b.create(0, 40)
    for k, (rule, aut) in enumerate([("fixed_indegree", False), ("fixed_outdegree", True),
                                     ("fixed_indegree", True), ("fixed_outdegree", False)]):
        for K in (1, 2, 7, 31, 32, 33, 100):
            src, tgt = (a, c) if k % 2 == 0 else (c, a)
            b.connect([src], [tgt], {"rule": rule, "n": K, "autapses": aut, "multapses": False}, SYN_N)
        b.connect([d], [a], {"rule": "fixed_indegree", "n": 5, "autapses": True, "multapses": True}, SYN_N)
        for p, src, tgt in ((0.3, d, d), (0.01, a, c), (1.0, d, a), (0.2, a, a)):
            b.connect([src], [tgt], {"rule": "pairwise_bernoulli", "p": p, "autapses": k % 2 == 1}, SYN_N)
    b.connect([a], [a], {"rule": "fixed_indegree", "n": 20, "autapses": False, "multapses": False}, SYN_N)
    b.connect([d], [d], {"rule": "fixed_outdegree", "n": 39, "autapses": False, "multapses": False}, SYN_N)
    return b.script("batch_mix")


def test_batched_floyd_and_bernoulli():
    # per call and as one batch (small-degree sampling and Bernoulli writing inside the batch's
    # fused launch): the oracle's connections, in generation order and after Prepare
    import paper_2512_09502_amd as snnc
    s = _batch_mix_script()
    compare_all(s, 0)
    net = snnc.Network(1, 0, s["seed"], s["dt"])
    reqs = []
    for op in s["ops"]:
        if op[0] == "create":
            net.create(op[1], op[2])
        else:
            reqs.append(op[1:])
    assert all(status == 0 for status, _ in net.submit_many(reqs))
    net.flush()
    ref = oracle.run_script(s, 0)
    for k in ("gen_src", "gen_tgt", "gen_delay", "gen_weight", "call_off"):   # generation order, per call
        compare(k, net.array(k), ref.array(k), s["name"] + " batched")
    net.prepare()
    for k in ("src", "tgt", "delay", "weight", "row_ptr"):
        compare(k, net.array(k), ref.array(k), s["name"] + " batched")
    net.close()


def test_first_occurrence_tuning_keys_reject_out_of_range():
    import paper_2512_09502_amd as snnc
    net = snnc.Network(1, 0, 1, 0.1)
    for key, bad in [("total_small_max", (1 << 15) + 1), ("total_small_max", -1), ("total_hash_max", (1 << 32) + 1)]:
        with pytest.raises(snnc.SnncError) as e:
            net.tune(key, bad)
        assert e.value.code == -1
    net.tune("total_small_max", 0)
    net.tune("total_hash_max", 1 << 32)
    net.close()
