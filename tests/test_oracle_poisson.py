"""Pins for the oracle's POISSON work function (the paper's framework probe, Section
6.3.2): the counter-based generator against its published known-answer vectors, the
exponential against the C library, and the deviates' distribution."""
import math
import os

import numpy as np
import pytest

from oracle import ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    n = 0
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        assert ref.philox4x32_10(v[0:4], v[4:6]) == v[6:10]
        n += 1
    assert n == 3


def test_expneg_within_two_ulp():
    xs = np.concatenate([np.linspace(0, 500, 20001), np.random.default_rng(0).uniform(0, 500, 20000)])
    worst = 0
    for x in xs:
        a = ref.expneg(float(x))
        b = math.exp(-float(x))
        worst = max(worst, abs(a - b) / math.ulp(b))
    assert worst <= 2.0, worst


@pytest.mark.parametrize("mu", [0.5, 5.0, 24.3, 137.0])
def test_poisson_moments(mu):
    n = 200_000
    d = ref.poisson(np.full(n, mu, np.float32), seed=12345)
    assert (d == np.round(d)).all() and d.min() >= 0
    m, v = d.mean(), d.var()
    assert abs(m - mu) < 5 * math.sqrt(mu / n)
    assert abs(v - mu) < 5 * mu * math.sqrt(2.0 / n) + 0.01
    if mu == 0.5:
        assert abs((d == 0).mean() - math.exp(-0.5)) < 0.005


def test_poisson_edge_means_and_seeds():
    x = np.array([0.0, -3.0, np.nan, 1e-30, 500.0, 1e9], np.float32)
    d = ref.poisson(x, seed=7)
    assert d[0] == 0 and d[1] == 0 and d[2] == 0 and d[3] == 0
    assert 400 < d[4] < 600 and 400 < d[5] < 600        # means clamp to 500
    a = ref.poisson(np.full(1000, 24.3, np.float32), seed=1)
    b = ref.poisson(np.full(1000, 24.3, np.float32), seed=1)
    c = ref.poisson(np.full(1000, 24.3, np.float32), seed=2)
    assert (a == b).all() and (a != c).any()
