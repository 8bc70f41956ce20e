"""Seeded synthetic inputs: instance lists for batched generation and
request streams for serving.  This module only draws parameters (numpy's
generator); it contains none of the generator's arithmetic.  Per-instance
seeds come from a caller-supplied function (the library's
kg_instance_seed, or the oracle's), so both sides use the same inputs.
"""
import json
import math
import os
from dataclasses import dataclass

import numpy as np

GNM, GNP = 0, 1


@dataclass
class Spec:
    n: int
    model: int
    directed: bool
    m: int
    p: float
    seed: int
    chunks: int

    def slots(self):
        return self.n * (self.n - 1) // (1 if self.directed else 2)

    def expected_edges(self):
        return self.m if self.model == GNM else self.p * self.slots()


POLICY_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "chunk_policy.json")
_policy = None


def policy_key(model, directed, ln, ld):
    """Key of the chunk-count table for floor(log2 n) = ln and
    floor(log2 degree) = ld; degree is the mean out-degree (directed) or the
    mean degree (undirected)."""
    return "%s/%s/%d/%d" % ("gnm" if model == GNM else "gnp", "d" if directed else "u", ln, ld)


def load_policy(path=None):
    """The persisted chunk-count table (written by `python -m
    paper_1710_07565_amd.tune --chunk-policy`)."""
    global _policy
    if path is None and _policy is not None:
        return _policy
    with open(path or POLICY_PATH) as f:
        tab = json.load(f)
    if path is None:
        _policy = tab
    return tab


def chunk_policy(model, directed, n, degree, table=None):
    """The paper's P for an instance of a batch or a request: looked up in
    the persisted table by (model, directed, floor(log2 n), floor(log2
    degree)), both logarithms clamped to the table's ranges.  The output
    bits depend on P, so it comes from this fixed table (not from timing on
    the machine at hand) and is recorded in the instance; P never exceeds n."""
    tab = table or load_policy()
    lo_n, hi_n = tab["log2n"]
    lo_d, hi_d = tab["log2d"]
    ln = min(max(int(math.floor(math.log2(max(int(n), 1)))), lo_n), hi_n)
    ld = min(max(int(math.floor(math.log2(max(float(degree), 1.0)))), lo_d), hi_d)
    P = int(tab["P"][policy_key(model, directed, ln, ld)])
    return max(1, min(P, int(n)))


def policy_cells(log2n=(10, 24), log2d=(1, 6)):
    """Every key of the table: both models, both directions, floor(log2 n) in
    log2n and floor(log2 degree) in log2d (inclusive)."""
    out = []
    for model in (GNM, GNP):
        for directed in (True, False):
            for ln in range(log2n[0], log2n[1] + 1):
                for ld in range(log2d[0], log2d[1] + 1):
                    out.append((model, directed, ln, ld))
    return out


def policy_probe(model, directed, ln, ld, count=4, rng_seed=7, seed_fn=None, base_seed=5):
    """Seeded instances inside one table cell (n in [2^ln, 2^(ln+1)), degree
    in [2^ld, 2^(ld+1)) capped at 64), without P: the tuner times them under
    every candidate P."""
    rng = np.random.default_rng([rng_seed, model, int(directed), ln, ld])
    out = []
    for i in range(count):
        n = int(2.0 ** rng.uniform(ln, ln + 1))
        d = min(float(2.0 ** rng.uniform(ld, ld + 1)), 64.0)
        seed = seed_fn(base_seed, i) if seed_fn else (base_seed * 1000003 + i)
        out.append((n, d, seed))
    return out


def make_instance(n, d, directed, model, seed, P=None):
    """An instance of mean degree d (the m and p rules of the batched and
    served workloads); P from the chunk-count table unless given."""
    N = n * (n - 1) // (1 if directed else 2)
    if P is None:
        P = chunk_policy(model, directed, n, d)
    if model == GNM:
        m = int(round(n * d if directed else n * d / 2.0))
        return Spec(n, GNM, directed, min(m, N), 0.0, seed, P)
    p = min(1.0, d / (n - 1))
    return Spec(n, GNP, directed, 0, p, seed, P)


def batch_instances(count=4096, base_seed=1, seed_fn=None, log2n=(10, 22), degree=(2.0, 64.0), rng_seed=20240101):
    """Uneven instances: n log-uniform in [2^a, 2^b], mean degree uniform,
    half directed, half G(n,m); seeds seed_fn(base_seed, i)."""
    rng = np.random.default_rng(rng_seed)
    out = []
    for i in range(count):
        n = int(2.0 ** rng.uniform(log2n[0], log2n[1]))
        d = float(rng.uniform(degree[0], degree[1]))
        directed = bool(rng.uniform() < 0.5)
        model = GNM if rng.uniform() < 0.5 else GNP
        seed = seed_fn(base_seed, i) if seed_fn else (base_seed * 1000003 + i)
        out.append(make_instance(n, d, directed, model, seed))
    return out


def request_stream(rate_per_s=2000.0, duration_s=60.0, base_seed=1, seed_fn=None, log2n=(12, 24),
                   degree=(4.0, 32.0), rng_seed=1):
    """Open-loop Poisson arrivals: (arrival time in s, Spec) pairs.  Equal mix
    of G(n,m) / G(n,p) and of directed / undirected."""
    rng = np.random.default_rng(rng_seed)
    t = 0.0
    out = []
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate_per_s))
        if t >= duration_s:
            break
        n = int(2.0 ** rng.uniform(log2n[0], log2n[1]))
        d = float(rng.uniform(degree[0], degree[1]))
        directed = bool(rng.uniform() < 0.5)
        model = GNM if rng.uniform() < 0.5 else GNP
        seed = seed_fn(base_seed, i) if seed_fn else (base_seed * 1000003 + i)
        out.append((t, make_instance(n, d, directed, model, seed)))
        i += 1
    return out
