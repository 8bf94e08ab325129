"""The seeded workload generators (parameter draws only): determinism, the
ranges each field is drawn from, the arrival rate, and the pooled-parameter
variant of the served stream."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_1905_03525_amd import workloads


def test_batch_instances_ranges_and_determinism():
    a = workloads.batch_instances(64)
    assert a == workloads.batch_instances(64)
    for i, p in enumerate(a):
        assert 10 <= p["k"] <= 24 and p["edge_factor"] in (4, 8, 16, 32)
        assert p["m"] == p["edge_factor"] << p["k"] and p["seed"] == i and p["table_bound"] == 0
        q = (p["a"], p["b"], p["c"], p["d"])
        assert min(q) >= 0.0 and abs(sum(q) - 1.0) < 1e-12


@pytest.mark.parametrize("reading", ["A", "B"])
def test_served_stream_fields(reading):
    reqs = workloads.served_requests(rate=2000.0, duration=2.0, reading=reading)
    # Poisson count: mean 4000, standard deviation about 63
    assert abs(len(reqs) - 4000) < 5 * math.sqrt(4000)
    ts = [p["t_arrival"] for p in reqs]
    assert ts == sorted(ts) and ts[-1] < 2.0
    for r, p in enumerate(reqs):
        assert p["id"] == r and p["seed"] == r and 12 <= p["k"] <= 28
        assert p["m"] in (8 << p["k"], 16 << p["k"]) and p["table_bound"] == 4096
    ks = np.array([p["k"] for p in reqs])
    if reading == "A":  # k uniform: every value about equally often
        counts = np.bincount(ks, minlength=29)[12:]
        assert counts.min() > 0.6 * counts.mean()
    else:               # ln k uniform: small k more frequent than large k
        assert np.mean(ks <= 20) > 0.55


def test_served_pool_repeats_parameter_sets():
    plain = workloads.served_requests(rate=2000.0, duration=1.0)
    pooled = workloads.served_requests(rate=2000.0, duration=1.0, pool=16)
    assert len(plain) == len(pooled)
    sets = {(p["a"], p["b"], p["c"], p["d"]) for p in pooled}
    assert len(sets) == 16            # ~2000 draws cover all 16 sets
    for p, q in zip(plain, pooled):   # arrivals, k and edge factor drawn before the parameters
        assert (p["t_arrival"], p["k"], p["m"]) == (q["t_arrival"], q["k"], q["m"])
    assert len({(p["a"], p["b"], p["c"], p["d"]) for p in plain}) == len(plain)
    with pytest.raises(ValueError):
        workloads.served_requests(duration=0.1, pool=-1)
