"""Oracle parity on the grid lengths of the large configurations.

The transforms are compiled per grid length: up to 128 points the x and y
passes run in one plane kernel, above that as an x pass plus a y line pass;
the z pass, the k-space factors and the inverse z pass run in one fused
kernel at every length; the wave sampler's inverse transform runs the z line
pass on its own.  So each of 128, 192, 256, 384 and 512 is its own code path
and each is compared here with the FP64 oracle.  N = 100 spheres in a box of
side L = 24 with the splitting parameter set to xi = 0.5 keep the oracle's
direct wave-vector sum near 4e4 vectors at every grid (the Gaussian's width
in grid units, hence the quadrature error, does not depend on the grid
spacing, and the truncation at the Nyquist wave number is far below eps).
Bars as everywhere: block error < eps = 1e-3 and per-particle error < 4 eps,
in both precisions.
"""
import functools

import numpy as np
import pytest

from gpu_common import PARTICLE_TOL, block_errors, dev, host, packing, particle_errors
from oracle import brownian, ewald
from paper_1709_06946_amd import inputs

pytestmark = pytest.mark.gpu

GRIDS = [128, 192, 256, 384, 512]
N, XI, TOL = 100, 0.5, 1e-3
PHI = 4.0 * np.pi * N / (3.0 * 24.0**3)
SEED = inputs.SEED_BASE + 51
KMAX = 2 * XI * np.sqrt(50.0)          # the oracle's wave-sum truncation


@functools.lru_cache(maxsize=None)
def system():
    x, L = packing(N, PHI, SEED)
    q = np.random.default_rng(SEED + 1).normal(size=(N, 11))
    return x, L, q


@functools.lru_cache(maxsize=None)
def oracle_product(stresslets_only=False):
    x, L, q = system()
    if stresslets_only:
        q = q.copy()
        q[:, 0:6] = 0.0
    return ewald.real_apply(x, q, L, XI), ewald.wave_apply(x, q, L, XI)


def _handle(grid, precision, **kw):
    from paper_1709_06946_amd import pse
    x, L, _ = system()
    h = pse.PSE(N, L, grid=grid, xi=XI, tol=1e-3, precision=precision, **kw)
    assert h.derived.grid == grid and abs(h.derived.xi - XI) < 1e-15
    return h


def _check(tag, y, ref):
    errs, perr = block_errors(y, ref), particle_errors(y, ref)
    print(tag, errs, perr, flush=True)
    assert max(errs.values()) < TOL, errs
    assert max(perr.values()) < PARTICLE_TOL, perr


@pytest.mark.parametrize('precision', [0, 1])
@pytest.mark.parametrize('grid', GRIDS)
def test_product_on_grid(grid, precision):
    """Wave part alone and the total product M q, every block."""
    import torch
    from paper_1709_06946_amd import pse
    x, L, q = system()
    r, w = oracle_product()
    h = _handle(grid, precision)
    try:
        out = torch.zeros((N, 11), dtype=torch.float64, device='cuda:0')
        h.mobility_apply(dev(x), dev(q), out, pse.PSE_WAVE)
        _check(f'g{grid} p{precision} wave', host(out), w)
        h.mobility_apply(dev(x), dev(q), out, pse.PSE_REAL | pse.PSE_WAVE)
        _check(f'g{grid} p{precision} total', host(out), r + w)
    finally:
        h.close()


@pytest.mark.parametrize('gridding', [1, 2])
@pytest.mark.parametrize('precision', [0, 1])
@pytest.mark.parametrize('grid', GRIDS)
def test_constraint_operator_on_grid(grid, precision, gridding):
    """The constraint operator M_ES (stresslets in, strains out) with the
    five moments gridded (1) or the Gaussian's gradient (2)."""
    import torch
    from paper_1709_06946_amd import pse
    x, L, q = system()
    r, w = oracle_product(stresslets_only=True)
    h = _handle(grid, precision, deriv_gridding=gridding)
    try:
        assert h.derived.deriv_gridding == gridding
        out = torch.zeros((N, 11), dtype=torch.float64, device='cuda:0')
        h.mobility_apply(dev(x), dev(q), out, pse.PSE_REAL | pse.PSE_WAVE | pse.PSE_ES_BLOCK)
        e = host(out)[:, 6:11]
        ref = (r + w)[:, 6:11]
        err = np.linalg.norm(e - ref) / np.linalg.norm(ref)
        d = np.linalg.norm(e - ref, axis=1).max() / np.sqrt(np.mean(np.sum(ref**2, axis=1)))
        print(f'g{grid} p{precision} dg{gridding} ES', err, d, flush=True)
        assert err < TOL and d < PARTICLE_TOL
    finally:
        h.close()


def _wave_noise(grid):
    """Wave noise on the canonical modes with |k| <= KMAX (zero elsewhere):
    the host array for the oracle and the same values on the device."""
    import torch
    x, L, _ = system()
    kap, idx = brownian.grid_half_space(grid, KMAX * L / (2 * np.pi))
    rng = np.random.default_rng(SEED + grid)
    vals = (rng.normal(size=(3, len(idx))) + 1j * rng.normal(size=(3, len(idx)))) * np.sqrt(0.5)
    shape = (3, grid, grid, grid // 2 + 1)
    host_psi = np.zeros(shape, complex)
    host_psi[:, idx[:, 0], idx[:, 1], idx[:, 2]] = vals
    dev_psi = torch.zeros(shape, dtype=torch.complex128, device='cuda:0')
    ii = [torch.as_tensor(idx[:, k], device='cuda:0') for k in range(3)]
    dev_psi[:, ii[0], ii[1], ii[2]] = torch.as_tensor(vals, device='cuda:0')
    return host_psi, dev_psi


@pytest.mark.parametrize('precision', [0, 1])
@pytest.mark.parametrize('grid', GRIDS)
def test_wave_sampler_on_grid(grid, precision):
    """M_w^(1/2) psi with the same noise: noise scaling, projection, the
    inverse z line pass and x-y transform, interpolation."""
    import torch
    x, L, _ = system()
    host_psi, dev_psi = _wave_noise(grid)
    ref = brownian.wave_sample(x, host_psi, L, grid, XI, kmax=KMAX)
    h = _handle(grid, precision)
    try:
        out = torch.zeros((N, 11), dtype=torch.float64, device='cuda:0')
        h.brownian_sample(dev(x), psi_wave=dev_psi, out_wave=out)
        _check(f'g{grid} p{precision} wave sampler', host(out), ref)
    finally:
        h.close()
        del dev_psi
        torch.cuda.empty_cache()
