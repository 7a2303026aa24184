"""Pins of the oracle's counter-based random numbers."""
import os

import numpy as np

from oracle import rng as R

HERE = os.path.dirname(__file__)


def test_splitmix64_published_sequence():
    want = [int(l, 16) for l in open(os.path.join(HERE, "golden", "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    state, got = 0, []
    for _ in range(len(want)):
        # generator form: advance the state by the golden increment, output mix(state);
        # splitmix64(x) = mix(x + increment), so output k is splitmix64(k * increment)
        got.append(R.splitmix64(state))
        state = (state + R.GOLDEN) & R.M64
    assert got == want


def test_u24_range_and_exact_float32():
    vals = [R.draw_u24(5, 1, 2, i, R.P_MUTATION, 7) for i in range(2000)]
    assert all(0 <= v < (1 << 24) for v in vals)
    u = np.array([R.uniform(5, 1, 2, i, R.P_MUTATION, 7) for i in range(2000)])
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_uniformity_chi_square():
    u = np.array([R.uniform(11, 0, 3, i, R.P_TOURNAMENT, 2) for i in range(20000)])
    counts, _ = np.histogram(u, bins=20, range=(0, 1))
    chi2 = float(((counts - 1000.0) ** 2 / 1000.0).sum())
    assert chi2 < 45.0          # 19 dof, p ~ 1e-3
    assert abs(u.mean() - 0.5) < 0.01


def test_coordinates_are_independent_streams():
    base = [R.draw_u24(3, 0, 0, 0, R.P_INIT, i) for i in range(64)]
    for field in range(5):
        coords = [0, 0, 0, R.P_INIT, 0]
        coords[field] += 1
        other = [R.draw_u24(3, *coords[:4], coords[4] + i) for i in range(64)]
        assert sum(a == b for a, b in zip(base, other)) <= 1


def test_randint_exact_range():
    n = 151
    vals = [R.randint(n, 9, 0, 1, i, R.P_TOURNAMENT, 0) for i in range(5000)]
    assert min(vals) >= 0 and max(vals) < n
    assert len(set(vals)) > 140
