"""Pins of the oracle's primitives against published values, closed forms and
distributions: Philox4x32-10, the uniform index map, the Box-Muller weight and
the delay-step distribution."""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert oracle.philox(ctr, key).tolist() == expect


def test_philox_counter_and_key_sensitivity():
    base = oracle.philox([1, 2, 3, 4], [5, 6])
    # every counter or key word changes the block (no word is ignored)
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] ^= 1
        assert oracle.philox(c, [5, 6]).tolist() != base.tolist()
    for i in range(2):
        k = [5, 6]
        k[i] ^= 1
        assert oracle.philox([1, 2, 3, 4], k).tolist() != base.tolist()


def test_philox_output_bits_are_balanced():
    # 4096 blocks on consecutive counters: each of the 128 output bits is set
    # about half the time (a round with a dropped term fails this badly)
    words = np.array([oracle.philox([i, 0, 0, 0], [1, 0]) for i in range(4096)], dtype=np.uint64)
    for w in range(4):
        for b in range(32):
            frac = float(((words[:, w] >> np.uint64(b)) & np.uint64(1)).mean())
            assert abs(frac - 0.5) < 5 * 0.5 / math.sqrt(4096)


# ----------------------------------------------------------------- index map
@pytest.mark.parametrize("n", [1, 2, 3, 7, 1000, 130000, 2**31 - 1, 2**32 + 5, 2**63 + 11])
def test_uniform_index_bounds(n):
    assert oracle.uniform_index(0, 0, n) == 0
    assert oracle.uniform_index(0xFFFFFFFF, 0xFFFFFFFF, n) == n - 1


def test_uniform_index_defining_inequality():
    # idx is the unique integer with idx * 2^64 <= u * n < (idx + 1) * 2^64
    rng = np.random.default_rng(5)
    for _ in range(2000):
        lo, hi = (int(x) for x in rng.integers(0, 2**32, size=2))
        n = int(rng.integers(1, 2**62))
        u = (hi << 32) | lo
        idx = oracle.uniform_index(lo, hi, n)
        assert idx * 2**64 <= u * n < (idx + 1) * 2**64


def test_uniform_index_power_of_two_is_top_bits():
    rng = np.random.default_rng(6)
    for _ in range(500):
        lo, hi = (int(x) for x in rng.integers(0, 2**32, size=2))
        k = int(rng.integers(0, 64))
        u = (hi << 32) | lo
        assert oracle.uniform_index(lo, hi, 2**k) == u >> (64 - k)


def test_uniform_index_is_monotone_in_u():
    n = 12345
    us = sorted(int(x) for x in np.random.default_rng(7).integers(0, 2**63, size=400))
    idx = [oracle.uniform_index(u & 0xFFFFFFFF, u >> 32, n) for u in us]
    assert idx == sorted(idx)


# ----------------------------------------------------------------- weights
def test_normal_weight_distribution():
    rng = np.random.default_rng(8)
    w0 = rng.integers(0, 2**32, size=40000, dtype=np.uint64)
    w1 = rng.integers(0, 2**32, size=40000, dtype=np.uint64)
    mean, sd = -0.5, 0.05
    x = np.array([oracle.normal_weight(int(a), int(b), mean, sd) for a, b in zip(w0, w1)])
    n = x.size
    assert abs(x.mean() - mean) < 5 * sd / math.sqrt(n)
    assert abs(x.std() - sd) < 5 * sd / math.sqrt(2 * n)
    assert stats.kstest((x - mean) / sd, "norm").pvalue > 1e-4


def test_normal_weight_special_words():
    # u1 = 1 (w0 = 2^32 - 1): the radius is 0, the weight is the mean in fp32
    for mean in (0.1, -0.5, 3.25):
        assert oracle.normal_weight(0xFFFFFFFF, 12345, mean, 0.7) == np.float32(mean)
    # half a turn apart the cosine flips sign: z(w1 + 2^31) = -z(w1)
    for w0, w1 in [(7, 11), (123456789, 2**30 - 3), (2**31, 99)]:
        a = oracle.normal_weight(w0, w1, 0.0, 1.0)
        b = oracle.normal_weight(w0, w1 + 2**31, 0.0, 1.0)
        assert abs(a + b) <= 4 * np.spacing(np.float32(abs(a)))
    # the radius is a Rayleigh variable: P(|z| at w1 = 0 <= r) = 1 - exp(-r^2 / 2)
    rng = np.random.default_rng(9)
    r = np.array([oracle.normal_weight(int(a), 0, 0.0, 1.0) for a in rng.integers(0, 2**32, size=20000)])
    assert (r >= 0).all()
    assert stats.kstest(r, "rayleigh").pvalue > 1e-4


# ----------------------------------------------------------------- delays
@pytest.mark.parametrize("mean,sd,lo", [(1.5, 0.75, 0.1), (3.0, 1.5, 0.1), (0.5, 2.0, 0.3), (10.0, 0.05, 0.1)])
def test_delay_table_matches_discretised_normal(mean, sd, lo):
    dt = 0.1
    klo, tab = oracle.delay_table(mean, sd, lo, dt)
    assert klo == round(lo / dt)
    # P(step <= k) for k = klo, klo+1, ... is P(d < (k + 1/2) dt), with the
    # mass below the clip folded into klo; thresholds are ceil(F 2^32)
    ks = klo + np.arange(tab.size)
    F = stats.norm.cdf(((ks + 0.5) * dt - mean) / sd)
    assert np.all(np.abs(tab / 2.0**32 - F) <= 2.0**-32 + 1e-12)
    assert np.all(np.diff(tab.astype(np.int64)) >= 0)
    # the table stops where the CDF reaches 1 at 32-bit resolution
    F_next = stats.norm.cdf(((ks[-1] + 1.5) * dt - mean) / sd)
    assert F_next > 1 - 2.0**-31


def test_delay_table_rejects_too_long():
    assert oracle.delay_table(7000.0, 1.0, 0.1, 0.1) is None


def test_delay_samples_chi_square():
    # sample the step distribution through a network: one Bernoulli p = 1
    # call gives n_s * n_t connections with independent SYN draws
    net = oracle.OracleNet(1, 0, 77, 0.1)
    a = net.create(0, 300)
    d = {"kind": "normal", "mean": 1.5, "sd": 0.75, "lo": 0.1}
    net.connect([a], [a], {"rule": "pairwise_bernoulli", "p": 1.0}, {"weight": {"kind": "const", "mean": 1.0}, "delay": d})
    steps = net.array("gen_delay").astype(np.int64)
    assert steps.size == 90000
    klo, tab = oracle.delay_table(1.5, 0.75, 0.1, 0.1)
    edges = np.concatenate([[0], tab.astype(np.float64), [2.0**32]]) / 2.0**32
    probs = np.diff(edges)
    counts = np.bincount(steps - klo, minlength=probs.size)
    assert counts.size == probs.size
    keep = probs * steps.size >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(probs[keep], probs[~keep].sum()) * steps.size
    assert stats.chisquare(obs, exp).pvalue > 1e-4


def test_constant_delay_steps():
    # 1.5 ms at dt = 0.1 ms is 15 steps; a delay below one step is rejected
    net = oracle.OracleNet(1, 0, 1, 0.1)
    a = net.create(0, 10)
    net.connect([a], [a], {"rule": "one_to_one"}, {"weight": {"kind": "const", "mean": 2.0},
                                                   "delay": {"kind": "const", "mean": 1.5}})
    assert set(net.array("gen_delay").tolist()) == {15}
    assert set(net.array("gen_weight").tolist()) == {2.0}
    with pytest.raises(oracle.OracleError):
        net.connect([a], [a], {"rule": "one_to_one"}, {"weight": {"kind": "const", "mean": 2.0},
                                                       "delay": {"kind": "const", "mean": 0.04}})
