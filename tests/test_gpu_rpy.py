"""RPY-level (forces-only) PSE on the same kernels, through the C ABI,
against the FP64 oracle: the product M_UF F (real and wave parts), its
equality with the force-velocity block of the full product, and the
Euler-Maruyama step with the split sampler restricted to the UF block, all
on the parity configurations (N = 100, phi = 0.1 and 0.01, 32^3, eps = 1e-3)
with the same noise on both sides.  The bar is the method tolerance 1e-3."""
import functools

import numpy as np
import pytest

from gpu_common import dev, host, packing, rel_err
from oracle import ewald, integrator
from paper_1709_06946_amd import inputs

pytestmark = pytest.mark.gpu

CASES = {
    'phi0.1': dict(N=100, phi=0.1, grid=32, seed=inputs.SEED_BASE + 30),
    'phi0.01': dict(N=100, phi=0.01, grid=32, seed=inputs.SEED_BASE + 37),
}
TOL = 1e-3


@functools.lru_cache(maxsize=None)
def case(name, precision=0, lanczos_tol=1e-3):
    from paper_1709_06946_amd import pse
    c = CASES[name]
    x, L = packing(c['N'], c['phi'], c['seed'])
    h = pse.PSE(c['N'], L, grid=c['grid'], tol=1e-3, precision=precision,
                lanczos_tol=lanczos_tol)
    F = np.random.default_rng(c['seed'] + 1).normal(size=(c['N'], 3))
    return h, x, L, F


def _rpy(h, x, F, parts):
    import torch
    out = torch.zeros((h.n, 3), dtype=torch.float64, device='cuda:0')
    h.rpy_apply(dev(x), dev(F), out, parts)
    return host(out)


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('precision', [0, 1])
def test_rpy_product_matches_oracle(name, precision):
    from paper_1709_06946_amd import pse
    h, x, L, F = case(name, precision)
    xi = h.derived.xi
    q = np.zeros((h.n, 11))
    q[:, 0:3] = F
    ref_real = ewald.real_apply(x, q, L, xi)[:, 0:3]
    ref_wave = ewald.wave_apply(x, q, L, xi)[:, 0:3]
    errs = dict(real=rel_err(_rpy(h, x, F, pse.PSE_REAL), ref_real),
                wave=rel_err(_rpy(h, x, F, pse.PSE_WAVE), ref_wave),
                total=rel_err(_rpy(h, x, F, pse.PSE_REAL | pse.PSE_WAVE), ref_real + ref_wave))
    print(name, precision, 'rpy product', errs)
    assert max(errs.values()) < TOL, errs


@pytest.mark.parametrize('name', list(CASES))
def test_rpy_product_is_force_velocity_block_of_full_product(name):
    """Three gridded components give the same U as the 11-component product
    with zero torques and stresslets (FP64: the same arithmetic up to
    rounding)."""
    import torch
    from paper_1709_06946_amd import pse
    h, x, L, F = case(name)
    q = np.zeros((h.n, 11))
    q[:, 0:3] = F
    full = torch.zeros((h.n, 11), dtype=torch.float64, device='cuda:0')
    h.mobility_apply(dev(x), dev(q), full, pse.PSE_REAL | pse.PSE_WAVE)
    err = rel_err(_rpy(h, x, F, pse.PSE_REAL | pse.PSE_WAVE), host(full)[:, 0:3])
    print(name, 'rpy vs full UF rows', err)
    assert err < 1e-12


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('precision', [0, 1])
def test_rpy_step_same_noise(name, precision):
    import torch
    h, x, L, F = case(name, precision, lanczos_tol=1e-8)
    c = CASES[name]
    g = h.derived.grid
    psi1 = np.random.default_rng(c['seed'] + 5).normal(size=(h.n, 3))
    psi2 = inputs.wave_noise(g, c['seed'] + 6)
    dt = 1e-3
    xt = dev(x)
    slip = torch.zeros((h.n, 3), dtype=torch.float64, device='cuda:0')
    U = torch.zeros((h.n, 3), dtype=torch.float64, device='cuda:0')
    rc, st = h.rpy_step(xt, dev(F), dt, psi_real=dev(psi1), psi_wave=dev(psi2), slip=slip,
                        velocity=U)
    ref = integrator.rpy_step(x, F, psi1, psi2, dt, L, g, h.derived.xi, xi_total=7.0 / L)
    x1 = host(xt)
    dx = x1 - x
    dx -= L * np.rint(dx / L)
    errs = dict(slip=rel_err(host(slip), ref['slip']), U=rel_err(host(U), ref['U']),
                dx=rel_err(dx, ref['dx']))
    print(name, precision, 'rpy step', errs, st)
    assert rc == 0 and st['converged'] == 1
    assert max(errs.values()) < TOL, errs
    assert np.all((x1 >= 0) & (x1 < L))


def test_rpy_step_internal_noise():
    """With Philox noise and no force the step is a pure Brownian move: finite,
    inside the box, reproducible for the same (seed, step) and different for
    another step."""
    import torch
    h, x, L, _ = case('phi0.1')
    moves = []
    for step in (3, 3, 4):
        xt = dev(x)
        rc, st = h.rpy_step(xt, None, 1e-3, seed=11, step=step)
        assert rc == 0 and st['converged'] == 1
        d = host(xt) - x
        d -= L * np.rint(d / L)
        moves.append(d)
    assert np.all(np.isfinite(moves[0])) and np.abs(moves[0]).max() > 0
    assert np.array_equal(moves[0], moves[1])
    assert not np.allclose(moves[0], moves[2])
