"""The synthetic input generators: non-overlapping packings at the requested
volume fraction (no part of the method lives here)."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1709_06946_amd import inputs


@pytest.mark.parametrize('phi', [0.05, 0.3])
def test_random_packings_are_non_overlapping(phi):
    x, L = inputs.packing(500, phi, seed=8)
    d, _ = cKDTree(x, boxsize=L).query(x, k=2)
    assert d[:, 1].min() >= 2.0 - 1e-9


@pytest.mark.parametrize('phi', [0.1, 0.3, 0.45])
def test_compiled_packings_non_overlapping_at_phi(phi):
    N = 5000
    x, L = inputs.packing(N, phi, seed=7)
    assert x.shape == (N, 3) and np.all((x >= 0) & (x < L))
    assert abs(N * 4.0 / 3.0 * np.pi / L**3 - phi) < 1e-12
    d, _ = cKDTree(x, boxsize=L).query(x, k=2)
    assert d[:, 1].min() >= 2.0


def test_compiled_packings_are_seeded_and_random():
    x1, L = inputs.packing(4000, 0.45, seed=11)
    x2, _ = inputs.packing(4000, 0.45, seed=11)
    x3, _ = inputs.packing(4000, 0.45, seed=12)
    assert np.array_equal(x1, x2) and not np.allclose(x1, x3)
    # a random (not crystalline) packing: the nearest-neighbour distances
    # spread over a range, and the positions fill the box uniformly
    d, _ = cKDTree(x1, boxsize=L).query(x1, k=2)
    assert np.percentile(d[:, 1], 90) - np.percentile(d[:, 1], 10) > 0.05
    counts = np.histogram(x1[:, 0], bins=8, range=(0, L))[0]
    assert counts.min() > 0.8 * 4000 / 8
