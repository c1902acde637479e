"""Stage-level checks of the HIP kernels through the C ABI diagnostics:
the 3D FFT against numpy's FFT and the Gaussian spreading/interpolation
against a direct numpy evaluation of the same sums."""
import numpy as np
import pytest

from gpu_common import dev, host, packing

pytestmark = pytest.mark.gpu


def _handle(N, L, grid, precision=0, **kw):
    from paper_1709_06946_amd import pse
    return pse.PSE(N, L, grid=grid, tol=1e-3, precision=precision, **kw)


@pytest.mark.parametrize('grid', [32, 48, 64, 96])
@pytest.mark.parametrize('direction', [-1, 1])
def test_fft3d_matches_numpy(grid, direction):
    import torch
    h = _handle(16, 5.0 * grid / 8, grid)
    rng = np.random.default_rng(grid)
    a = rng.normal(size=(3, grid, grid, grid)) + 1j * rng.normal(size=(3, grid, grid, grid))
    t = dev(a, torch.complex128)
    h.fft3d(t, direction)
    ref = (np.fft.fftn(a, axes=(1, 2, 3)) if direction < 0
           else np.fft.ifftn(a, axes=(1, 2, 3)) * grid**3)
    err = np.abs(host(t) - ref).max() / np.abs(ref).max()
    assert err < 1e-13, err


def test_fft3d_mixed_precision():
    import torch
    grid = 64
    h = _handle(16, 40.0, grid, precision=1)
    rng = np.random.default_rng(3)
    a = rng.normal(size=(2, grid, grid, grid)) + 1j * rng.normal(size=(2, grid, grid, grid))
    t = dev(a, torch.complex128)
    h.fft3d(t, -1)
    ref = np.fft.fftn(a, axes=(1, 2, 3))
    err = np.abs(host(t) - ref).max() / np.abs(ref).max()
    assert err < 3e-6, err


def _gauss_weights(h, x):
    d = h.derived
    P, hh, ng = d.support, d.h, d.grid
    kcoef = 2 * d.xi**2 / d.eta_s
    knorm = np.sqrt(2 * d.xi**2 / (np.pi * d.eta_s))
    f = x / hh
    start = (np.floor(f + 0.5).astype(int) - (P - 1) // 2 if P % 2
             else np.floor(f).astype(int) - P // 2 + 1)
    idx = start[:, :, None] + np.arange(P)[None, None, :]          # (N,3,P)
    dist = idx * hh - x[:, :, None]
    w = knorm * np.exp(-kcoef * dist**2)                            # (N,3,P)
    return idx % ng, w


def _spread_ref(h, x, q):
    ng = h.derived.grid
    idx, w = _gauss_weights(h, x)
    out = np.zeros((q.shape[1], ng, ng, ng))
    for p in range(x.shape[0]):
        W = np.einsum('a,b,c->cba', w[p, 0], w[p, 1], w[p, 2])     # (z,y,x)
        iz, iy, ix = np.ix_(idx[p, 2], idx[p, 1], idx[p, 0])
        for c in range(q.shape[1]):
            np.add.at(out[c], (iz, iy, ix), W * q[p, c])
    return out


def _interp_ref(h, x, g):
    idx, w = _gauss_weights(h, x)
    out = np.zeros((x.shape[0], g.shape[0]))
    for p in range(x.shape[0]):
        W = np.einsum('a,b,c->cba', w[p, 0], w[p, 1], w[p, 2])
        iz, iy, ix = np.ix_(idx[p, 2], idx[p, 1], idx[p, 0])
        out[p] = (g[:, iz, iy, ix] * W[None]).sum(axis=(1, 2, 3))
    return out


@pytest.mark.parametrize('ncomp', [1, 5, 11])
@pytest.mark.parametrize('precision', [0, 1])
def test_spread_and_interpolate(ncomp, precision):
    import torch
    x, L = packing(100, 0.1, 21)
    h = _handle(100, L, 32, precision=precision)
    rng = np.random.default_rng(ncomp)
    q = rng.normal(size=(100, ncomp))
    g = torch.zeros((ncomp, 32, 32, 32), dtype=torch.float64, device='cuda:0')
    h.spread(dev(x), dev(q), g)
    ref = _spread_ref(h, x, q)
    tol = 1e-12 if precision == 0 else 2e-6
    assert np.abs(host(g) - ref).max() < tol * np.abs(ref).max()
    field = rng.normal(size=(ncomp, 32, 32, 32))
    out = torch.zeros((100, ncomp), dtype=torch.float64, device='cuda:0')
    h.interpolate(dev(x), dev(field), out)
    ref = _interp_ref(h, x, field)
    assert np.abs(host(out) - ref).max() < tol * np.abs(ref).max()


def test_spread_handles_positions_outside_box():
    """Positions are wrapped into [0, L): shifting by lattice vectors does not
    change the spread grid."""
    import torch
    x, L = packing(100, 0.1, 22)
    h = _handle(100, L, 32)
    q = np.random.default_rng(1).normal(size=(100, 3))
    g1 = torch.zeros((3, 32, 32, 32), dtype=torch.float64, device='cuda:0')
    g2 = torch.zeros_like(g1)
    h.spread(dev(x), dev(q), g1)
    shift = L * np.random.default_rng(2).integers(-3, 4, size=(100, 3))
    h.spread(dev(x + shift), dev(q), g2)
    assert np.abs(host(g1) - host(g2)).max() < 1e-12 * np.abs(host(g1)).max()


@pytest.mark.parametrize('precision', [0, 1])
@pytest.mark.parametrize('grid', [32, 96, 128, 192, 256, 384])
@pytest.mark.parametrize('direction', [-1, 1])
def test_rfft3d_matches_numpy(grid, direction, precision):
    """The real transforms of the product and the sampler (plane kernel up to
    128, x pass + line passes above; half spectra with the kx = Ng/2 column
    not stored) against numpy's rfftn / irfftn."""
    import torch
    nc = 2
    h = _handle(16, 5.0 * grid / 8, grid, precision=precision)
    rng = np.random.default_rng(grid + 7 * (direction > 0))
    a = rng.normal(size=(nc, grid, grid, grid))
    spec = np.fft.rfftn(a, axes=(1, 2, 3))
    spec[..., grid // 2] = 0.0
    if direction < 0:
        src = a
        ref = spec[..., :grid // 2]
    else:
        src = np.ascontiguousarray(spec[..., :grid // 2]).view(np.float64)
        ref = np.fft.irfftn(spec, s=(grid, grid, grid), axes=(1, 2, 3)) * grid**3
    t = dev(np.ascontiguousarray(src).reshape(nc, grid, grid, grid))
    h.rfft3d(t, direction)
    out = host(t)
    if direction < 0:
        out = out.view(np.complex128).reshape(nc, grid, grid, grid // 2)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print(grid, direction, precision, err)
    assert err < (1e-12 if precision == 0 else 5e-6), err
    h.close()
