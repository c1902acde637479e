"""The synthetic input generators: non-overlapping packings at the requested
volume fraction (no part of the method lives here)."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1709_06946_amd import inputs


@pytest.mark.parametrize('phi', [0.1, 0.3, 0.45])
def test_jittered_lattice_is_non_overlapping_at_phi(phi):
    N = 3000
    x, L = inputs.jittered_lattice(N, phi, seed=7)
    assert x.shape == (N, 3) and np.all((x >= 0) & (x < L))
    assert abs(N * 4.0 / 3.0 * np.pi / L**3 - phi) < 1e-12
    d, _ = cKDTree(x, boxsize=L).query(x, k=2)
    assert d[:, 1].min() >= 2.0


@pytest.mark.parametrize('phi', [0.05, 0.3])
def test_random_packings_are_non_overlapping(phi):
    x, L = inputs.packing(500, phi, seed=8)
    d, _ = cKDTree(x, boxsize=L).query(x, k=2)
    assert d[:, 1].min() >= 2.0 - 1e-9


def test_large_packings_use_the_lattice():
    x, L = inputs.packing(inputs.LATTICE_N, 0.1, seed=9)
    assert x.shape == (inputs.LATTICE_N, 3)
