"""Pins of the oracle's connection rules: exact counts the rules fix (K per
target or source, N in total, one-to-one pairs), the autapse and multapse
flags, and the outcome distributions by brute-force enumeration on tiny sets
(chi-square against the exact probabilities)."""
import itertools
import math
from collections import Counter

import numpy as np
import pytest
from scipy import stats

import oracle

SYN = {"weight": {"kind": "const", "mean": 1.0}, "delay": {"kind": "const", "mean": 0.1}}


def _chi2_ok(counts: Counter, probs: dict, n: int, pmin=1e-4):
    keys = list(probs)
    assert set(counts) <= set(keys), f"impossible outcomes {set(counts) - set(keys)}"
    if len(keys) == 1:
        return counts[keys[0]] == n
    obs = np.array([counts.get(k, 0) for k in keys], float)
    exp = np.array([probs[k] * n for k in keys], float)
    return stats.chisquare(obs, exp).pvalue > pmin


def _many_calls(n_s, n_t, conn, reps, seed=3):
    """reps identical calls on one host; S = first n_s neurons, T = first n_t
    (so S and T overlap).  Returns per-call generation-order sources/targets."""
    net = oracle.OracleNet(1, 0, seed, 0.1)
    net.create(0, max(n_s, n_t))
    S, T = [(0, 0, n_s)], [(0, 0, n_t)]
    for _ in range(reps):
        net.connect(S, T, conn, SYN)
    src = net.array("gen_src").astype(np.int64)
    tgt = net.array("gen_tgt").astype(np.int64)
    return src, tgt


CASES_K = [(n_s, n_t, K, aut, mult)
           for n_s in (2, 3, 4) for n_t in (1, 3) for K in (1, 2, 3)
           for aut in (True, False) for mult in (True, False)
           if mult or K <= n_s - (0 if aut else 1)]


@pytest.mark.parametrize("n_s,n_t,K,aut,mult", CASES_K)
def test_indegree_enumeration(n_s, n_t, K, aut, mult):
    reps = 2000
    conn = {"rule": "fixed_indegree", "n": K, "autapses": aut, "multapses": mult}
    src, tgt = _many_calls(n_s, n_t, conn, reps)
    per_call = n_t * K
    assert src.size == reps * per_call                 # exactly K per target
    src = src.reshape(reps, n_t, K)
    tgt = tgt.reshape(reps, n_t, K)
    assert (tgt == np.arange(n_t)[None, :, None]).all()
    cand = [s for s in range(n_s) if aut or s != 0]    # target 0 is neuron 0
    if mult:
        probs = {t: 1.0 / len(cand) ** K for t in itertools.product(cand, repeat=K)}
    else:
        subsets = list(itertools.combinations(cand, K))
        probs = {t: 1.0 / len(subsets) for t in subsets}
        assert (np.diff(src, axis=2) > 0).all()        # distinct, ascending
    if not aut:
        assert (src != np.arange(n_t)[None, :, None]).all()
    counts = Counter(tuple(int(x) for x in row) for row in src[:, 0, :])
    assert _chi2_ok(counts, probs, reps)


@pytest.mark.parametrize("n_s,n_t,K,aut,mult", [(n_t, n_s, K, aut, mult) for (n_s, n_t, K, aut, mult) in CASES_K])
def test_outdegree_enumeration(n_s, n_t, K, aut, mult):
    reps = 2000
    conn = {"rule": "fixed_outdegree", "n": K, "autapses": aut, "multapses": mult}
    src, tgt = _many_calls(n_s, n_t, conn, reps)
    assert src.size == reps * n_s * K                  # exactly K per source
    src = src.reshape(reps, n_s, K)
    tgt = tgt.reshape(reps, n_s, K)
    assert (src == np.arange(n_s)[None, :, None]).all()
    cand = [t for t in range(n_t) if aut or t != 0]
    if mult:
        probs = {t: 1.0 / len(cand) ** K for t in itertools.product(cand, repeat=K)}
    else:
        subsets = list(itertools.combinations(cand, K))
        probs = {t: 1.0 / len(subsets) for t in subsets}
    if not aut:
        assert (tgt != np.arange(n_s)[None, :, None]).all()
    counts = Counter(tuple(int(x) for x in row) for row in tgt[:, 0, :])
    assert _chi2_ok(counts, probs, reps)


@pytest.mark.parametrize("aut,mult", [(True, True), (False, True), (True, False), (False, False)])
def test_total_number_enumeration(aut, mult):
    n_s, n_t, N, reps = 2, 2, 2, 3000
    conn = {"rule": "fixed_total_number", "n": N, "autapses": aut, "multapses": mult}
    src, tgt = _many_calls(n_s, n_t, conn, reps)
    assert src.size == reps * N                         # exactly N in total
    pairs = list(zip(src.reshape(reps, N).tolist(), tgt.reshape(reps, N).tolist()))
    valid = [(s, t) for s in range(n_s) for t in range(n_t) if aut or s != t]
    outcomes = []
    for ss, tt in pairs:
        pr = tuple(zip(ss, tt))
        assert all(p in valid for p in pr)
        outcomes.append(tuple(sorted(pr)) if not mult else pr)
        if not mult:
            assert len(set(pr)) == N
    if mult:
        probs = {t: 1.0 / len(valid) ** N for t in itertools.product(valid, repeat=N)}
    else:
        subsets = list(itertools.combinations(valid, N))
        probs = {t: 1.0 / len(subsets) for t in subsets}
    assert _chi2_ok(Counter(outcomes), probs, reps)


def test_total_number_exact_and_uniform():
    net = oracle.OracleNet(1, 0, 11, 0.1)
    a = net.create(0, 50)
    b = net.create(0, 40)
    N = 60000
    net.connect([a], [b], {"rule": "fixed_total_number", "n": N}, SYN)
    s, t = net.array("gen_src"), net.array("gen_tgt")
    assert s.size == N and s.max() < 50
    assert (t >= 50).all() and (t < 90).all()
    cells = np.bincount(s.astype(np.int64) * 40 + (t.astype(np.int64) - 50), minlength=2000)
    assert stats.chisquare(cells).pvalue > 1e-4
    # candidates are consumed in order: element indices are 0..N-1
    assert (net.array("gen_e") == np.arange(N)).all()


@pytest.mark.parametrize("aut,mult", [(True, True), (False, True), (True, False), (False, False)])
def test_total_number_over_several_hosts(aut, mult):
    """Targets on three hosts: the hosts' shares together are exactly the first
    N valid candidates of the same rule on one host holding all neurons (same
    ordinals, same draws), and each host keeps the ones it holds."""
    N, sizes = 700, [30, 45, 25]
    conn = {"rule": "fixed_total_number", "n": N, "autapses": aut, "multapses": mult}
    shares = []
    for pl in range(3):
        net = oracle.OracleNet(3, pl, 17, 0.1)
        pops = [net.create(h, n) for h, n in enumerate(sizes)]
        net.connect(pops, pops, conn, SYN)
        shares.append((net.array("gen_e"), net.array("gen_src"), net.array("gen_tgt")))
    one = oracle.OracleNet(1, 0, 17, 0.1)
    pop = one.create(0, sum(sizes))
    one.connect([pop], [pop], conn, SYN)
    e1, s1, t1 = one.array("gen_e"), one.array("gen_src"), one.array("gen_tgt")
    assert e1.size == N
    e_all = np.concatenate([sh[0] for sh in shares])
    assert np.array_equal(np.sort(e_all), e1)
    first = np.cumsum([0] + sizes)
    for pl, (e, s, t) in enumerate(shares):
        idx = np.searchsorted(e1, e)
        assert (s == s1[idx]).all()
        assert (t + first[pl] == t1[idx]).all()           # same target, as a local id of host pl
        assert ((t1 >= first[pl]) & (t1 < first[pl + 1])).sum() == e.size


@pytest.mark.parametrize("p", [0.0, 0.03, 0.5, 1.0])
def test_bernoulli_count_band(p):
    net = oracle.OracleNet(1, 0, 21, 0.1)
    a = net.create(0, 300)
    net.connect([a], [a], {"rule": "pairwise_bernoulli", "p": p, "autapses": True}, SYN)
    n = 300 * 300
    k = net.array("gen_src").size
    pp = math.floor(p * 2**32) / 2**32 if p < 1 else 1.0
    sigma = math.sqrt(n * pp * (1 - pp))
    assert abs(k - n * pp) <= 5 * sigma + 1e-9


def test_bernoulli_pairs_and_autapses():
    reps, n = 400, 6
    net = oracle.OracleNet(1, 0, 5, 0.1)
    a = net.create(0, n)
    for _ in range(reps):
        net.connect([a], [a], {"rule": "pairwise_bernoulli", "p": 0.3, "autapses": False}, SYN)
    s = net.array("gen_src").astype(np.int64)
    t = net.array("gen_tgt").astype(np.int64)
    assert (s != t).all()
    cells = np.bincount(t * n + s, minlength=n * n).reshape(n, n)
    off = cells[~np.eye(n, dtype=bool)]
    pp = math.floor(0.3 * 2**32) / 2**32
    assert np.all(np.abs(off - reps * pp) <= 5 * math.sqrt(reps * pp * (1 - pp)))
    # target-major element order: e = t * n_s + s, increasing within a call
    e = net.array("gen_e").astype(np.int64)
    assert (e == t * n + s).all()


def test_one_to_one_closed_form():
    net = oracle.OracleNet(1, 0, 1, 0.1)
    a = net.create(0, 20)
    b = net.create(0, 20)
    net.connect([a], [b], {"rule": "one_to_one"}, SYN)
    assert (net.array("gen_src") == np.arange(20)).all()
    assert (net.array("gen_tgt") == np.arange(20, 40)).all()
    net.connect([a], [a], {"rule": "one_to_one", "autapses": False}, SYN)   # all autapses: none
    assert net.array("gen_src").size == 20
    net.connect([(0, 0, 10)], [(0, 5, 10)], {"rule": "one_to_one", "autapses": False}, SYN)
    assert net.array("gen_src").size == 30
    with pytest.raises(oracle.OracleError):
        net.connect([a], [(0, 0, 5)], {"rule": "one_to_one"}, SYN)


def test_indegree_exact_and_outdegree_mean():
    net = oracle.OracleNet(1, 0, 1, 0.1)
    a = net.create(0, 1000)
    b = net.create(0, 500)
    K = 100
    net.connect([a], [b], {"rule": "fixed_indegree", "n": K}, SYN)
    s, t = net.array("gen_src").astype(np.int64), net.array("gen_tgt").astype(np.int64)
    assert (np.bincount(t - 1000, minlength=500) == K).all()
    assert s.min() >= 0 and s.max() < 1000
    outdeg = np.bincount(s, minlength=1000)
    mu = K * 500 / 1000
    assert abs(outdeg.mean() - mu) < 1e-9       # total is exact
    # each source's out-degree is Binomial(K * n_t, 1 / n_s)
    var = K * 500 * (1 / 1000) * (1 - 1 / 1000)
    assert abs(outdeg.var() - var) < 5 * var * math.sqrt(2 / 1000)


def test_invalid_specs_rejected():
    net = oracle.OracleNet(2, 0, 1, 0.1)
    a = net.create(0, 5)
    with pytest.raises(oracle.OracleError):       # K > candidates without multapses
        net.connect([a], [a], {"rule": "fixed_indegree", "n": 5, "autapses": False, "multapses": False}, SYN)
    with pytest.raises(oracle.OracleError):       # segment outside the created range
        net.connect([(0, 3, 5)], [a], {"rule": "fixed_indegree", "n": 1}, SYN)
    with pytest.raises(oracle.OracleError):       # overlapping segments in one set
        net.connect([(0, 0, 3), (0, 2, 2)], [a], {"rule": "fixed_indegree", "n": 1}, SYN)
    with pytest.raises(oracle.OracleError):       # p outside [0, 1]
        net.connect([a], [a], {"rule": "pairwise_bernoulli", "p": 1.5}, SYN)
    net.connect([a], [a], {"rule": "fixed_indegree", "n": 4, "autapses": False, "multapses": False}, SYN)


def _bern_threshold(p):
    return 2**32 if p >= 1 else math.floor(p * 2**32)


@pytest.mark.parametrize("n_s,n_t,p,aut", [(5, 3, 0.3, True), (3, 4, 0.5, False), (7, 2, 0.1, True)])
def test_bernoulli_pair_enumeration(n_s, n_t, p, aut):
    """Brute force over many calls on tiny sets: every pair connects with
    probability T_p / 2^32 (chi-square per pair), the outcomes of the four
    pairs that share a Philox block are jointly independent (chi-square over
    the 16 joint outcomes), and so are neighbouring pairs across block and
    target boundaries (p^2).  n_s not a multiple of 4 puts pairs of two targets
    in one block."""
    reps = 3000
    net = oracle.OracleNet(1, 0, 17, 0.1)
    a = net.create(0, max(n_s, n_t))
    for _ in range(reps):
        net.connect([(0, 0, n_s)], [(0, 0, n_t)], {"rule": "pairwise_bernoulli", "p": p, "autapses": aut}, SYN)
    s = net.array("gen_src").astype(np.int64)
    t = net.array("gen_tgt").astype(np.int64)
    e = net.array("gen_e").astype(np.int64)
    assert (e == t * n_s + s).all()                      # element index = target-major pair index
    net.prepare()
    off = net.array("call_off").astype(np.int64)         # first generated index of each call
    assert off.size == reps + 1
    call = np.repeat(np.arange(reps), np.diff(off))
    hit = np.zeros((reps, n_t * n_s), bool)
    hit[call, e] = True
    pp = _bern_threshold(p) / 2**32
    valid = np.array([aut or (q % n_s) != (q // n_s) for q in range(n_s * n_t)])
    assert not hit[:, ~valid].any()                      # autapses skipped when excluded
    freq = hit[:, valid].sum(0)
    sd = math.sqrt(reps * pp * (1 - pp))
    assert np.all(np.abs(freq - reps * pp) <= 5 * sd)
    assert stats.chisquare(freq, np.full(freq.size, freq.sum() / freq.size)).pvalue > 1e-4
    # joint outcomes of a whole block of four valid pairs
    for b in range(n_s * n_t // 4):
        qs = list(range(4 * b, 4 * b + 4))
        if not valid[qs].all():
            continue
        code = (hit[:, qs] * (1 << np.arange(4))).sum(1)
        obs = np.bincount(code, minlength=16)
        k = np.array([bin(c).count("1") for c in range(16)])
        exp = reps * pp ** k * (1 - pp) ** (4 - k)
        assert stats.chisquare(obs, exp).pvalue > 1e-4
    # neighbouring valid pairs q, q + 1 (inside a block, across blocks, across targets)
    pairs = [q for q in range(n_s * n_t - 1) if valid[q] and valid[q + 1]]
    both = sum(int((hit[:, q] & hit[:, q + 1]).sum()) for q in pairs)
    n_adj = reps * len(pairs)
    assert abs(both - n_adj * pp * pp) <= 5 * math.sqrt(n_adj * pp * pp * (1 - pp * pp))


@pytest.mark.parametrize("p", [0.0, 0.001, 0.25, 0.7, 1.0])
def test_bernoulli_pairs_recomputed_from_philox(p):
    """Per-pair recomputation on a random sample: pair q connects iff word
    (q mod 4) of the BERN block q / 4 (Philox4x32-10 pinned by its
    known-answer vectors) is below floor(p 2^32)."""
    n_s, n_t, seed = 123, 57, 29
    net = oracle.OracleNet(1, 0, seed, 0.1)
    a = net.create(0, n_s)
    b = net.create(0, n_t)
    net.connect([a], [a], {"rule": "fixed_indegree", "n": 1}, SYN)              # call 0 (other stream)
    net.connect([a], [b], {"rule": "pairwise_bernoulli", "p": p}, SYN)           # call 1
    e = net.array("gen_e").astype(np.int64)[n_s:]
    s = net.array("gen_src").astype(np.int64)[n_s:]
    t = net.array("gen_tgt").astype(np.int64)[n_s:] - n_s
    assert (e == t * n_s + s).all() and (np.diff(e) > 0).all()
    got = set(e.tolist())
    thr = _bern_threshold(p)
    rng = np.random.default_rng(4)
    sample = rng.choice(n_s * n_t, size=600, replace=False).tolist() + sorted(got)[:50]
    for q in sample:
        blk = q // 4
        w = oracle.philox([blk & 0xFFFFFFFF, blk >> 32, 2, 0], [seed, 1])
        assert (int(w[q % 4]) < thr) == (q in got), q
    if p == 1.0:
        assert len(got) == n_s * n_t
    if p == 0.0:
        assert not got


def test_bernoulli_element_replay_matches_generation():
    net = oracle.OracleNet(1, 0, 3, 0.1)
    a = net.create(0, 150)
    net.connect([a], [a], {"rule": "pairwise_bernoulli", "p": 0.1, "autapses": False}, SYN)
    e = set(net.array("gen_e").tolist())
    rng = np.random.default_rng(0)
    for q in rng.integers(0, 150 * 150, size=400).tolist() + sorted(e)[:100]:
        r = net.element(0, q)
        assert (r is not None) == (q in e)
