"""Seeded synthetic inputs: instance lists for batched generation and
request streams for serving.  This module only draws parameters (numpy's
generator); it contains none of the generator's arithmetic.  Per-instance
seeds come from a caller-supplied function (the library's
kg_instance_seed, or the oracle's), so both sides use the same inputs.
"""
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


def chunk_policy(model, directed, n, degree):
    """The paper's P for an instance in a batch (output bits depend on it, so
    it is recorded in the instance).  Directed instances use one row chunk:
    the tile tree already gives the GPU its parallelism.  Undirected ones use
    enough sections that rectangles (cheap to decode) carry most edges."""
    if directed:
        return 1
    if n < 2**8:
        return 1
    if n < 2**14:
        return 8
    return 32


def _instance(n, d, directed, model, seed):
    N = n * (n - 1) // (1 if directed else 2)
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
        out.append(_instance(n, d, directed, model, seed))
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
        out.append((t, _instance(n, d, directed, model, seed)))
        i += 1
    return out
