"""Seeded synthetic workload scripts.

A script is a plain dict ``{"P", "seed", "dt", "ops"}``; ``ops`` is a list of

* ``("create", host, n)`` -- Create(population, n) on a virtual host, and
* ``("connect", src_segments, tgt_segments, conn_spec, syn_spec, alpha)`` --
  Connect over node sets given as ``(host, first, n)`` segments (the position
  of a neuron in a set is its rank in the concatenation of the segments);
  ``alpha = -1`` marks point-to-point exchange, ``alpha >= 0`` a collective
  group.

The same script is replayed on every virtual host (the paper's premise that
all processes run the same script), by the GPU library and by the oracle
alike.  This module only makes structural choices (population sizes,
probabilities, in-degrees, request streams) with ``numpy`` generators seeded
per workload; it contains none of the construction arithmetic.

The workloads stand in for the paper's two models (the multi-area model, whose
connectivity data is not available here, and the scalable balanced network of
the HPC benchmark) with synthetic networks of the same shape.
"""
from __future__ import annotations

import math

import numpy as np

DT = 0.1          # ms, the paper's simulation resolution
SEED = 1          # Philox seed for every workload

W_E = {"kind": "normal", "mean": 0.1, "sd": 0.01}
W_I = {"kind": "normal", "mean": -0.5, "sd": 0.05}
D_CONST_15 = {"kind": "const", "mean": 1.5}


def _round_half_away(x: float) -> int:
    return int(math.floor(x + 0.5)) if x >= 0 else -int(math.floor(-x + 0.5))


class _Builder:
    def __init__(self, P: int, seed: int = SEED, dt: float = DT):
        self.P, self.seed, self.dt = P, seed, dt
        self.M = [0] * P
        self.ops = []

    def create(self, host: int, n: int) -> tuple:
        seg = (host, self.M[host], n)
        self.M[host] += n
        self.ops.append(("create", host, n))
        return seg

    def connect(self, src, tgt, conn, syn, alpha=-1):
        self.ops.append(("connect", [tuple(s) for s in src], [tuple(t) for t in tgt],
                         dict(conn), dict(syn), int(alpha)))

    def script(self, name: str, **info) -> dict:
        return {"name": name, "P": self.P, "seed": self.seed, "dt": self.dt,
                "ops": self.ops, "info": info}


def balanced_small(n_e: int = 800, n_i: int = 200, k_e: int = 80, k_i: int = 20) -> dict:
    """Balanced E/I network on one host: 1,000 neurons, fixed in-degree 100
    (80 E + 20 I), no autapses, delay 1.5 ms, normal weights; 1e5 connections."""
    b = _Builder(1)
    e = b.create(0, n_e)
    i = b.create(0, n_i)
    allset = [e, i]
    conn_e = {"rule": "fixed_indegree", "n": k_e, "autapses": False, "multapses": True}
    conn_i = {"rule": "fixed_indegree", "n": k_i, "autapses": False, "multapses": True}
    b.connect([e], allset, conn_e, {"weight": W_E, "delay": D_CONST_15})
    b.connect([i], allset, conn_i, {"weight": W_I, "delay": D_CONST_15})
    return b.script("balanced_1k_k100", conns=(n_e + n_i) * (k_e + k_i))


COLUMN_BASE = (20000, 5800, 22000, 5500, 4900, 1100, 14000, 2900)


def column8(scale: float = 1.0, seed: int = 1002) -> dict:
    """8-population cortical-column-shaped network on one host.  Sizes are
    seeded around 20k/5.8k/22k/5.5k/4.9k/1.1k/14k/2.9k (even index =
    excitatory); every ordered pair (i -> j) is one fixed-total-number call with
    N_ij = round(p_ij N_i N_j), p_ij ~ U(0.01, 0.15); autapses and multapses
    allowed; delays N(1.5, 0.75) ms clipped at 0.1 ms; weights by source type."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(8)
    p = rng.uniform(0.01, 0.15, size=(8, 8))
    sizes = [max(1, _round_half_away(base * scale * (1.0 + 0.05 * gi))) for base, gi in zip(COLUMN_BASE, g)]
    b = _Builder(1)
    pops = [b.create(0, n) for n in sizes]
    delay = {"kind": "normal", "mean": 1.5, "sd": 0.75, "lo": 0.1}
    total = 0
    for i in range(8):
        for j in range(8):
            n_ij = _round_half_away(p[i, j] * sizes[i] * sizes[j])
            total += n_ij
            conn = {"rule": "fixed_total_number", "n": n_ij, "autapses": True, "multapses": True}
            b.connect([pops[i]], [pops[j]], conn, {"weight": W_E if i % 2 == 0 else W_I, "delay": delay})
    return b.script("column8_total_number", conns=total, sizes=sizes, scale=scale)


def multiarea_p2p(P: int = 32, n_e: int = 104000, n_i: int = 26000, k_e: int = 2800, k_i: int = 700,
                  k_remote_max: int = 96, seed: int = 1003) -> dict:
    """One rank's view of a P-area model with point-to-point exchange.  Each
    host holds one area (E and I populations).  For each target host tau, the
    local E and I populations connect to all of tau's neurons with fixed
    in-degree (no autapses); then each other area sigma projects its E
    population onto tau with in-degree K ~ U{0..k_remote_max} (skipped when 0)."""
    rng = np.random.default_rng(seed)
    kr = rng.integers(0, k_remote_max + 1, size=(P, P))
    b = _Builder(P)
    E, I = [], []
    for h in range(P):
        E.append(b.create(h, n_e))
        I.append(b.create(h, n_i))
    d_local = {"kind": "normal", "mean": 1.5, "sd": 0.75, "lo": 0.1}
    d_remote = {"kind": "normal", "mean": 3.0, "sd": 1.5, "lo": 0.1}
    for tau in range(P):
        tgt = [E[tau], I[tau]]
        b.connect([E[tau]], tgt, {"rule": "fixed_indegree", "n": k_e, "autapses": False, "multapses": True},
                  {"weight": W_E, "delay": d_local})
        b.connect([I[tau]], tgt, {"rule": "fixed_indegree", "n": k_i, "autapses": False, "multapses": True},
                  {"weight": W_I, "delay": d_local})
        for sigma in range(P):
            if sigma == tau or kr[sigma, tau] == 0:
                continue
            b.connect([E[sigma]], tgt, {"rule": "fixed_indegree", "n": int(kr[sigma, tau]),
                                        "autapses": True, "multapses": True},
                      {"weight": W_E, "delay": d_remote}, alpha=-1)
    # connections held by each host: every target draws k_e + k_i local and sum_sigma K[sigma, tau] remote sources
    by_host = [(n_e + n_i) * (k_e + k_i + int(kr[:, tau].sum() - kr[tau, tau])) for tau in range(P)]
    return b.script("multiarea_p2p", k_remote=kr.tolist(), conns_by_host=by_host)


def balanced_collective(P: int = 1024, n_e: int = 160000, n_i: int = 40000, k_e: int = 9000,
                        k_i: int = 2250) -> dict:
    """One rank's share of the scalable balanced network (HPC-benchmark
    shaped) distributed over P hosts with collective exchange (group 0):
    E_all -> ALL_all with in-degree k_e and I_all -> ALL_all with k_i,
    autapses and multapses allowed, delay 1.5 ms, normal weights."""
    b = _Builder(P)
    E, I = [], []
    for h in range(P):
        E.append(b.create(h, n_e))
        I.append(b.create(h, n_i))
    allset = [(h, 0, n_e + n_i) for h in range(P)]
    b.connect(E, allset, {"rule": "fixed_indegree", "n": k_e, "autapses": True, "multapses": True},
              {"weight": W_E, "delay": D_CONST_15}, alpha=0)
    b.connect(I, allset, {"rule": "fixed_indegree", "n": k_i, "autapses": True, "multapses": True},
              {"weight": W_I, "delay": D_CONST_15}, alpha=0)
    return b.script("balanced_collective", conns_per_host=(n_e + n_i) * (k_e + k_i))


def balanced_indegree(in_scale: int = 2, P: int = 1024, n_e: int = 160000, n_i: int = 40000, k_e: int = 9000,
                      k_i: int = 2250, group: int = 0) -> dict:
    """The balanced network with an in-degree scale (the paper's in-degree
    appendix): each host holds n_e / s excitatory and n_i / s inhibitory
    neurons, every neuron receives s * k_e excitatory and s * k_i inhibitory
    connections, and the weights are divided by s, so the connections per
    host stay (n_e + n_i) (k_e + k_i) while the sources (and images) shrink
    by s."""
    s = int(in_scale)
    ne, ni = max(1, n_e // s), max(1, n_i // s)
    b = _Builder(P)
    E, I = [], []
    for h in range(P):
        E.append(b.create(h, ne))
        I.append(b.create(h, ni))
    allset = [seg for h in range(P) for seg in (E[h], I[h])]
    w_e = {"kind": "normal", "mean": W_E["mean"] / s, "sd": W_E["sd"] / s}
    w_i = {"kind": "normal", "mean": W_I["mean"] / s, "sd": W_I["sd"] / s}
    b.connect(E, allset, {"rule": "fixed_indegree", "n": k_e * s, "autapses": True, "multapses": True},
              {"weight": w_e, "delay": D_CONST_15}, group)
    b.connect(I, allset, {"rule": "fixed_indegree", "n": k_i * s, "autapses": True, "multapses": True},
              {"weight": w_i, "delay": D_CONST_15}, group)
    return b.script(f"balanced_indegree_x{s}", conns=(ne + ni) * (k_e + k_i) * s, in_scale=s)


def served_requests(n_requests: int = 10000, n_pops: int = 64, pop_min: int = 1000, pop_max: int = 200000,
                    size_min: float = 1e2, size_max: float = 1e7, seed: int = 1005) -> dict:
    """A stream of Connect requests of uneven size on one host: 64
    populations with log-uniform sizes in [1e3, 2e5]; request sizes S
    log-uniform in [1e2, 1e7]; rule uniform over the five rules; source and
    target populations uniform; autapse and multapse flags coin flips.
    in-degree: n_t = min(N_t, S) targets, K = max(1, S // n_t); out-degree:
    the mirror; total number: N = S; one-to-one: n = min(S, N_s, N_t);
    Bernoulli: p ~ U(0.001, 0.2) on the first n_t = min(N_t, ceil(sqrt(S/p)))
    targets and n_s = min(N_s, ceil(S / (p n_t))) sources.  No parameter
    is trimmed to what the library accepts: a degree above the candidates or
    a total number above the pairs without multapses is invalid, a degree
    above the library's limit without multapses unsupported, and the library
    rejects such requests (the stream goes on).  Poisson arrival times for
    an offered rate of one request per unit time are in info['arrival']."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(pop_min), math.log(pop_max), size=n_pops)).astype(np.int64)
    b = _Builder(1)
    pops = [b.create(0, int(n)) for n in sizes]
    rules = ["fixed_indegree", "fixed_outdegree", "fixed_total_number", "pairwise_bernoulli", "one_to_one"]
    delay = {"kind": "normal", "mean": 1.5, "sd": 0.75, "lo": 0.1}
    offered = 0
    for _ in range(n_requests):
        S = int(math.exp(rng.uniform(math.log(size_min), math.log(size_max))))
        rule = rules[int(rng.integers(0, 5))]
        i, j = int(rng.integers(0, n_pops)), int(rng.integers(0, n_pops))
        aut, mult = bool(rng.integers(0, 2)), bool(rng.integers(0, 2))
        h, fi, Ni = pops[i]
        _, fj, Nj = pops[j]
        conn = {"rule": rule, "autapses": aut, "multapses": mult}
        if rule == "fixed_indegree":
            nt = min(Nj, S)
            K = max(1, S // nt)
            src, tgt, conn["n"] = [(h, fi, Ni)], [(h, fj, nt)], K
            offered += nt * K
        elif rule == "fixed_outdegree":
            ns = min(Ni, S)
            K = max(1, S // ns)
            src, tgt, conn["n"] = [(h, fi, ns)], [(h, fj, Nj)], K
            offered += ns * K
        elif rule == "fixed_total_number":
            N = S
            src, tgt, conn["n"] = [(h, fi, Ni)], [(h, fj, Nj)], N
            offered += N
        elif rule == "one_to_one":
            n = min(S, Ni, Nj)
            src, tgt = [(h, fi, n)], [(h, fj, n)]
            offered += n
        else:
            p = float(rng.uniform(0.001, 0.2))
            nt = min(Nj, int(math.ceil(math.sqrt(S / p))))
            ns = min(Ni, int(math.ceil(S / (p * nt))))
            src, tgt, conn["p"] = [(h, fi, ns)], [(h, fj, nt)], p
            offered += int(p * ns * nt)
        b.connect(src, tgt, conn, {"weight": W_E if i % 2 == 0 else W_I, "delay": delay})
    arrival = np.cumsum(rng.exponential(1.0, size=n_requests)).tolist()
    return b.script("served_requests", offered=offered, arrival=arrival, pop_sizes=sizes.tolist())


def random_tiny(seed: int, P: int | None = None) -> dict:
    """A small random script mixing all rules, flags, groups and segment
    layouts over a few virtual hosts, for property and parity tests."""
    rng = np.random.default_rng(10_000 + seed)
    if P is None:
        P = int(rng.integers(1, 5))
    b = _Builder(P, seed=int(rng.integers(0, 2**32)), dt=0.1)
    pops = []
    for _ in range(int(rng.integers(2, 6))):
        h = int(rng.integers(0, P))
        pops.append(b.create(h, int(rng.integers(1, 40))))
    rules = ["one_to_one", "fixed_indegree", "fixed_outdegree", "fixed_total_number", "pairwise_bernoulli"]

    def pick_set():
        k = int(rng.integers(1, min(3, len(pops)) + 1))
        idx = rng.choice(len(pops), size=k, replace=False)
        segs = []
        for i in idx:
            h, f, n = pops[i]
            a = int(rng.integers(0, n))
            c = int(rng.integers(a + 1, n + 1))
            segs.append((h, f + a, c - a))
        return segs

    for _ in range(int(rng.integers(1, 8))):
        rule = rules[int(rng.integers(0, 5))]
        src, tgt = pick_set(), pick_set()
        ns, nt = sum(s[2] for s in src), sum(t[2] for t in tgt)
        aut, mult = bool(rng.integers(0, 2)), bool(rng.integers(0, 2))
        conn = {"rule": rule, "autapses": aut, "multapses": mult}
        if rule == "one_to_one":
            m = min(ns, nt)
            src, tgt = _truncate(src, m), _truncate(tgt, m)
        elif rule == "fixed_indegree":
            conn["n"] = int(rng.integers(0, max(1, ns - 1) + 1)) if not mult else int(rng.integers(0, 12))
        elif rule == "fixed_outdegree":
            conn["n"] = int(rng.integers(0, max(1, nt - 1) + 1)) if not mult else int(rng.integers(0, 12))
        elif rule == "fixed_total_number":
            conn["n"] = int(rng.integers(0, max(1, ns * nt // 2) + 1))
        else:
            conn["p"] = float(rng.choice([0.0, 0.05, 0.3, 0.7, 1.0]))
        wkind = "normal" if rng.integers(0, 2) else "const"
        w = {"kind": wkind, "mean": float(rng.normal()), "sd": 0.1}
        if rng.integers(0, 2):
            d = {"kind": "normal", "mean": float(rng.uniform(0.5, 3.0)), "sd": float(rng.uniform(0.1, 1.0)),
                 "lo": 0.1 * int(rng.integers(1, 4))}
        else:
            d = {"kind": "const", "mean": 0.1 * int(rng.integers(1, 40))}
        alpha = int(rng.integers(-1, 2))
        b.connect(src, tgt, conn, {"weight": w, "delay": d}, alpha)
    return b.script(f"random_tiny_{seed}")


def distributed_indegree_assigned(P: int = 4, n_per_host: int = 500, K: int = 20, seed: int = 1006) -> dict:
    """Fixed in-degree over populations distributed across hosts, built the
    way of the paper's distributed fixed in-degree subsection: every target
    host tau draws, for each of its targets, K sources uniformly from the
    whole distributed source population (triplets (sigma~, s~, t)), sorts the
    triplets by sigma~ and then s~, splits them by source host and connects
    each part with the assigned-nodes rule (one call per (tau, sigma)).  The
    structural draws come from numpy (seeded); the pairs are the calls'
    inputs.  E populations on every host are the sources, all neurons the
    targets; weights N(0.1, 0.01), delays N(1.5, 0.75) ms clipped at 0.1."""
    rng = np.random.default_rng(seed)
    b = _Builder(P, seed=1)
    pops = [b.create(h, n_per_host) for h in range(P)]
    delay = {"kind": "normal", "mean": 1.5, "sd": 0.75, "lo": 0.1}
    n_src = P * n_per_host
    for tau in range(P):
        t = np.repeat(np.arange(n_per_host, dtype=np.int64), K)
        g = rng.integers(0, n_src, size=t.size)            # global source index over the population
        sig, s = g // n_per_host, g % n_per_host
        order = np.lexsort((s, sig))                        # by sigma~, then s~ (stable)
        sig, s, t = sig[order], s[order], t[order]
        for sigma in range(P):
            m = sig == sigma
            if not m.any():
                continue
            conn = {"rule": "assigned_nodes", "pairs": (s[m].tolist(), t[m].tolist())}
            b.connect([pops[sigma]], [pops[tau]], conn, {"weight": W_E, "delay": delay})
    return b.script("distributed_indegree_assigned", K=K)


def random_assigned(seed: int, P: int | None = None) -> dict:
    """Random scripts with assigned-nodes calls (random pairs over random
    multi-host segment sets, groups -1..1) mixed with fixed in-degree calls,
    for property and parity tests."""
    rng = np.random.default_rng(20_000 + seed)
    if P is None:
        P = int(rng.integers(1, 5))
    b = _Builder(P, seed=int(rng.integers(0, 2**32)), dt=0.1)
    pops = [b.create(int(rng.integers(0, P)), int(rng.integers(1, 60))) for _ in range(int(rng.integers(2, 6)))]

    def pick_set():
        k = int(rng.integers(1, min(3, len(pops)) + 1))
        segs = []
        for i in rng.choice(len(pops), size=k, replace=False):
            h, f, n = pops[i]
            a = int(rng.integers(0, n))
            c = int(rng.integers(a + 1, n + 1))
            segs.append((h, f + a, c - a))
        return segs

    delay = {"kind": "normal", "mean": 1.5, "sd": 0.5, "lo": 0.1}
    for _ in range(int(rng.integers(1, 7))):
        src, tgt = pick_set(), pick_set()
        ns, nt = sum(x[2] for x in src), sum(x[2] for x in tgt)
        alpha = int(rng.integers(-1, 2))
        if rng.integers(0, 4) == 0:
            b.connect(src, tgt, {"rule": "fixed_indegree", "n": int(rng.integers(1, 6))}, {"weight": W_I, "delay": delay},
                      alpha)
            continue
        n = int(rng.integers(0, 300))
        pairs = (rng.integers(0, ns, size=n).tolist(), rng.integers(0, nt, size=n).tolist())
        b.connect(src, tgt, {"rule": "assigned_nodes", "pairs": pairs}, {"weight": W_E, "delay": delay}, alpha)
    return b.script(f"random_assigned_{seed}")


def _truncate(segs, m):
    out = []
    for h, f, n in segs:
        if m <= 0:
            break
        k = min(n, m)
        out.append((h, f, k))
        m -= k
    return out

