"""Seeded synthetic inputs: the instance lists of the batched and served
workloads.  Parameter draws only (numpy's default_rng); none of the
sampler's arithmetic lives here, so the HIP path and the CPU oracle can both
be fed from this module.

Batched workload: instance i draws, from default_rng(i), k uniform in
{10..24}, then an edge factor from {4, 8, 16, 32}, then (a, b, c, d) from
Dirichlet(4, 2, 2, 1); m = edge_factor * 2^k and the Philox seed is i.

Served workload: a Poisson stream (exponential gaps from
default_rng(arrival_seed)) at `rate` requests/s for `duration` s; request r
draws from default_rng(r) its k (reading "A": an integer uniform in
[12, 28], i.e. n log-uniform; reading "B": ln k uniform on [ln 12, ln 28],
rounded), an edge factor from {8, 16} and (a, b, c, d) from
Dirichlet(4, 2, 2, 1); its seed is r.  With a parameter pool of P sets
(drawn in order from default_rng(arrival_seed + 1)), request r instead
takes set j, j uniform in [0, P) drawn from default_rng(r) after its edge
factor, so that requests repeat tables.
"""
from __future__ import annotations

import math

import numpy as np

RMAT_VARIABLE = 1
DIRICHLET = (4.0, 2.0, 2.0, 1.0)


def dirichlet_q(rng: np.random.Generator) -> tuple:
    """(a, b, c, d) from Dirichlet(4, 2, 2, 1), d completing the sum to 1."""
    q = rng.dirichlet(DIRICHLET)
    a, b, c = float(q[0]), float(q[1]), float(q[2])
    return a, b, c, 1.0 - a - b - c


def batch_instances(n: int = 512, k_min: int = 10, k_max: int = 24, edge_factors=(4, 8, 16, 32)) -> list:
    """Instance dicts (a, b, c, d, k, path_mode, table_bound=0 for the
    autotuner, seed, edge_begin=0, m, edge_factor)."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(i)
        k = int(rng.integers(k_min, k_max + 1))
        ef = int(rng.choice(edge_factors))
        a, b, c, d = dirichlet_q(rng)
        out.append(dict(a=a, b=b, c=c, d=d, k=k, path_mode=RMAT_VARIABLE, table_bound=0, seed=i, edge_begin=0,
                        m=ef << k, edge_factor=ef))
    return out


def request_k(rng: np.random.Generator, reading: str, k_min: int = 12, k_max: int = 28) -> int:
    if reading == "A":
        return int(rng.integers(k_min, k_max + 1))
    if reading == "B":
        return int(round(math.exp(rng.uniform(math.log(k_min), math.log(k_max)))))
    raise ValueError(f"unknown reading {reading!r}")


def served_requests(rate: float = 2000.0, duration: float = 60.0, arrival_seed: int = 2019, reading: str = "A",
                    k_min: int = 12, k_max: int = 28, edge_factors=(8, 16), table_bound: int = 4096,
                    pool: int = 0) -> list:
    """Request dicts in arrival order: id, t_arrival (s), a, b, c, d, k,
    path_mode, table_bound, seed, edge_begin=0, m.  pool > 0 draws the
    parameters from that many pre-drawn sets."""
    if pool < 0:
        raise ValueError("pool must be >= 0")
    prng = np.random.default_rng(arrival_seed + 1)
    sets = [dirichlet_q(prng) for _ in range(pool)]
    gaps = np.random.default_rng(arrival_seed)
    t, out, r = 0.0, [], 0
    while True:
        t += float(gaps.exponential(1.0 / rate))
        if t >= duration:
            break
        rng = np.random.default_rng(r)
        k = request_k(rng, reading, k_min, k_max)
        ef = int(rng.choice(edge_factors))
        a, b, c, d = sets[int(rng.integers(pool))] if pool else dirichlet_q(rng)
        out.append(dict(id=r, t_arrival=t, a=a, b=b, c=c, d=d, k=k, path_mode=RMAT_VARIABLE,
                        table_bound=table_bound, seed=r, edge_begin=0, m=ef << k))
        r += 1
    return out
