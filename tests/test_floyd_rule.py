"""CPU check of the decision rule the GPU's parallel Floyd sampler uses
(csrc/gen.hip, k_floyd): with the same draws, (a) first occurrences found in
the sorted (value, step) keys, (b) links from a high draw to the step whose
fallback it is, resolved by pointer jumping, and (c) the chosen values listed
as the distinct low draws followed by the flagged positions of the top window
give exactly the sorted set of Robert Floyd's sequential insertion, on random
cases including degrees equal to the candidate count."""
import numpy as np
import pytest


def _sequential(n, K, r):
    chosen = set()
    for j in range(K):
        m = n - K + j
        chosen.add(m if r[j] in chosen else r[j])
    return sorted(chosen)


def _parallel_rule(n, K, r):
    base = n - K
    keys = sorted((r[j], j) for j in range(K))
    first = {}
    for v, j in keys:
        first.setdefault(v, j)
    dup = [1 if first[r[j]] < j else 0 for j in range(K)]
    link = [r[j] - base if r[j] >= base else j for j in range(K)]
    span = 1
    while span < K:
        dup = [dup[j] | dup[link[j]] for j in range(K)]
        link = [link[link[j]] for j in range(K)]
        span <<= 1
    flags = [0] * K
    for j in range(K):
        if dup[j]:
            flags[j] = 1
        elif r[j] >= base:
            flags[r[j] - base] = 1
    low = [keys[q][0] for q in range(K) if keys[q][0] < base and (q == 0 or keys[q - 1][0] != keys[q][0])]
    return low + [base + i for i in range(K) if flags[i]]


@pytest.mark.parametrize("seed", range(4))
def test_parallel_floyd_rule_equals_sequential_insertion(seed):
    rng = np.random.default_rng(seed)
    for _ in range(500):
        K = int(rng.integers(1, 70))
        n = K + int(rng.integers(0, 3)) if rng.integers(0, 4) == 0 else K + int(rng.integers(0, 200))
        r = [int(rng.integers(0, n - K + j + 1)) for j in range(K)]
        assert _parallel_rule(n, K, r) == _sequential(n, K, r), (n, K, r)
