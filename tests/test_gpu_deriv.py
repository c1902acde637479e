"""Derivative gridding (the couplets -- stresslets and torques -- spread
with the Gaussian's gradient onto three grids, rotation and strain
interpolated with it; forces and velocities on their moment grids) against
the FP64 oracle's Ewald sums: the constraint operator M_ES over the
tolerance sweep eps in {1e-2 ... 1e-5}, its wave-space part alone in both
precisions, the whole 11 x 11 product over the sweep and per input group,
agreement with moment gridding, and the constrained step with the same
noise.  The bar is the method tolerance eps of each configuration."""
import math

import numpy as np
import pytest

from gpu_common import dev, host, packing, rel_err
from oracle import ewald, integrator
from paper_1709_06946_amd import inputs

pytestmark = pytest.mark.gpu


def _min_xi(L, eps, a=1.0):
    # rcut = 2a + sqrt(ln(1/eps))/xi must not exceed L/3
    return 1.05 * math.sqrt(math.log(1.0 / eps)) / (L / 3.0 - 2.0 * a)


def _es(h, x, q, parts):
    import torch

    from paper_1709_06946_amd import pse
    out = torch.zeros((h.n, 11), dtype=torch.float64, device='cuda:0')
    h.mobility_apply(dev(x), dev(q), out, parts | pse.PSE_ES_BLOCK)
    return host(out)[:, 6:11]


def _stresslets(N, seed):
    q = np.zeros((N, 11))
    q[:, 6:11] = np.random.default_rng(seed).normal(size=(N, 5))
    return q


@pytest.mark.parametrize('eps', [1e-2, 1e-3, 1e-4, 1e-5])
@pytest.mark.parametrize('mode', [1, 2])
def test_es_block_within_tolerance(eps, mode):
    from paper_1709_06946_amd import pse
    x, L = packing(100, 0.1, inputs.SEED_BASE)
    h = pse.PSE(100, L, tol=eps, xi=_min_xi(L, eps), deriv_gridding=mode)
    d = h.derived
    # derivative gridding takes one more support point; at eps = 1e-5 that
    # exceeds 10 and the moment gridding is used
    assert d.deriv_gridding == (mode if eps >= 1e-4 else 1)
    q = _stresslets(100, 21)
    ref = (ewald.real_apply(x, q, L, d.xi) + ewald.wave_apply(x, q, L, d.xi))[:, 6:11]
    err = rel_err(_es(h, x, q, pse.PSE_REAL | pse.PSE_WAVE), ref)
    print(f'mode={mode} eps={eps:g} grid={d.grid} P={d.support} xi={d.xi:.3f}', err)
    assert err < eps


@pytest.mark.parametrize('phi', [0.1, 0.01])
@pytest.mark.parametrize('precision', [0, 1])
def test_es_wave_part_derivative(phi, precision):
    from paper_1709_06946_amd import pse
    x, L = packing(100, phi, inputs.SEED_BASE + 3)
    h = pse.PSE(100, L, grid=32, tol=1e-3, precision=precision, deriv_gridding=2)
    assert h.derived.deriv_gridding == 2
    q = _stresslets(100, 22)
    ref = ewald.wave_apply(x, q, L, h.derived.xi)[:, 6:11]
    err = rel_err(_es(h, x, q, pse.PSE_WAVE), ref)
    print(f'phi={phi} precision={precision} wave ES', err)
    assert err < 1e-3


def test_derivative_and_moment_gridding_agree_at_tight_tolerance():
    """Both quadratures of the same operator converge to the same sums: at
    eps = 1e-4 (derivative gridding at P = 10, its largest support) they
    agree to within twice the tolerance."""
    from paper_1709_06946_amd import pse
    x, L = packing(100, 0.1, inputs.SEED_BASE + 5)
    eps = 1e-4
    q = _stresslets(100, 23)
    out = {}
    for mode in (1, 2):
        h = pse.PSE(100, L, tol=eps, xi=_min_xi(L, eps), deriv_gridding=mode)
        assert h.derived.deriv_gridding == mode
        out[mode] = _es(h, x, q, pse.PSE_WAVE)
    err = rel_err(out[2], out[1])
    print('derivative vs moment gridding at eps=1e-4', err)
    assert err < 2e-4


@pytest.mark.parametrize('phi', [0.1, 0.01])
def test_step_with_derivative_gridding_same_noise(phi):
    import torch

    from paper_1709_06946_amd import pse
    x, L = packing(100, phi, inputs.SEED_BASE + 9)
    h = pse.PSE(100, L, grid=32, tol=1e-3, lanczos_tol=1e-8, gmres_tol=1e-8,
                deriv_gridding=2)
    g = h.derived.grid
    FL = inputs.forces_torques(100, inputs.SEED_BASE + 10)
    psi1 = inputs.real_noise(100, inputs.SEED_BASE + 11)
    psi2 = inputs.wave_noise(g, inputs.SEED_BASE + 12)
    dt = 1e-3
    xt = dev(x)
    S = torch.zeros((100, 5), dtype=torch.float64, device='cuda:0')
    rc, st = h.constrained_step(xt, dev(FL), dt, psi_real=dev(psi1), psi_wave=dev(psi2),
                                stresslet=S)
    ref = integrator.midpoint_step(x, FL, psi1, psi2, dt, L, g, h.derived.xi,
                                   xi_total=7.0 / L)
    dx = host(xt) - x
    dx -= L * np.rint(dx / L)
    errs = dict(S=rel_err(host(S), ref['S']), dx=rel_err(dx, ref['dx']))
    print(f'phi={phi} derivative gridding step', errs, st)
    assert rc == 0 and st['converged'] == 1
    assert max(errs.values()) < 1e-3, errs


# Derivative gridding of every wave-space product: forces on their moment
# grids, torques and stresslets together on the gradient grids, velocity
# interpolated plainly, rotation and strain from the gradient.

def _full(h, x, q, parts):
    import torch
    out = torch.zeros((h.n, 11), dtype=torch.float64, device='cuda:0')
    h.mobility_apply(dev(x), dev(q), out, parts)
    return host(out)


@pytest.mark.parametrize('eps', [1e-2, 1e-3, 1e-4])
def test_full_product_within_tolerance(eps):
    from gpu_common import block_errors, particle_errors
    from paper_1709_06946_amd import pse
    x, L = packing(100, 0.1, inputs.SEED_BASE + 31)
    h = pse.PSE(100, L, tol=eps, xi=_min_xi(L, eps), deriv_gridding=2)
    d = h.derived
    assert d.deriv_gridding == 2
    q = np.random.default_rng(32).normal(size=(100, 11))
    ref = ewald.real_apply(x, q, L, d.xi) + ewald.wave_apply(x, q, L, d.xi)
    y = _full(h, x, q, pse.PSE_REAL | pse.PSE_WAVE)
    be, pe = block_errors(y, ref), particle_errors(y, ref)
    print(f'eps={eps:g} grid={d.grid} P={d.support}', be, pe)
    assert max(be.values()) < eps, be
    assert max(pe.values()) < 4 * eps, pe


@pytest.mark.parametrize('group', ['F', 'L', 'S'])
@pytest.mark.parametrize('precision', [0, 1])
def test_wave_blocks_of_each_input_group(group, precision):
    """Each input group alone (forces, torques, stresslets) against the
    oracle's wave sums, every output block: a wrong sign or factor in one
    coupling (a torque column, a rotation row) shows in its own block."""
    from gpu_common import block_errors
    from paper_1709_06946_amd import pse
    x, L = packing(100, 0.1, inputs.SEED_BASE + 33)
    h = pse.PSE(100, L, grid=32, tol=1e-3, precision=precision, deriv_gridding=2)
    assert h.derived.deriv_gridding == 2
    cols = {'F': slice(0, 3), 'L': slice(3, 6), 'S': slice(6, 11)}[group]
    q = np.zeros((100, 11))
    q[:, cols] = np.random.default_rng(34).normal(size=(100, cols.stop - cols.start))
    ref = ewald.wave_apply(x, q, L, h.derived.xi)
    be = block_errors(_full(h, x, q, pse.PSE_WAVE), ref)
    print(f'group={group} precision={precision}', be)
    assert max(be.values()) < 2e-3, be


def test_derivative_and_moment_gridding_agree_on_the_full_product():
    """The two quadratures of the whole product converge to the same sums:
    at eps = 1e-4 they agree to within twice the tolerance, block by block."""
    from gpu_common import block_errors
    from paper_1709_06946_amd import pse
    x, L = packing(100, 0.1, inputs.SEED_BASE + 35)
    eps = 1e-4
    q = np.random.default_rng(36).normal(size=(100, 11))
    out = {}
    for mode in (1, 2):
        h = pse.PSE(100, L, tol=eps, xi=_min_xi(L, eps), deriv_gridding=mode)
        assert h.derived.deriv_gridding == mode
        out[mode] = _full(h, x, q, pse.PSE_WAVE)
    be = block_errors(out[2], out[1])
    print('derivative vs moment gridding, full product', be)
    assert max(be.values()) < 2e-4, be
