"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Inputs are seeded hard-sphere packings (N = 100, phi = 0.1 and 0.01 in a
32^3 grid, eps = 1e-3) with i.i.d. N(0, 1) moments and noise.  Every result is
compared block by block (U, Omega, E) by relative 2-norm error, with the
method tolerance eps = 1e-3 of the configuration as the bar, and particle by
particle (largest error over the RMS magnitude, bar 4 eps).  The FP64 and
the mixed-precision forms are both held to these bars against the FP64
oracle.
"""
import functools

import numpy as np
import pytest

from gpu_common import (PARTICLE_TOL, block_errors, dev, host, packing, particle_err,
                        particle_errors, rel_err)
from oracle import brownian, ewald, integrator
from paper_1709_06946_amd import inputs

pytestmark = pytest.mark.gpu

CASES = {
    'phi0.1': dict(N=100, phi=0.1, grid=32, seed=inputs.SEED_BASE),
    'phi0.01': dict(N=100, phi=0.01, grid=32, seed=inputs.SEED_BASE + 7),
}
TOL = 1e-3


@functools.lru_cache(maxsize=None)
def case(name, precision=0, lanczos_tol=1e-3, gmres_tol=1e-6):
    from paper_1709_06946_amd import pse
    c = CASES[name]
    x, L = packing(c['N'], c['phi'], c['seed'])
    h = pse.PSE(c['N'], L, grid=c['grid'], tol=1e-3, precision=precision,
                lanczos_tol=lanczos_tol, gmres_tol=gmres_tol)
    return h, x, L


@functools.lru_cache(maxsize=None)
def moments(name):
    c = CASES[name]
    return np.random.default_rng(c['seed'] + 11).normal(size=(c['N'], 11))


@functools.lru_cache(maxsize=None)
def oracle_parts(name):
    h, x, L = case(name)
    q = moments(name)
    xi = h.derived.xi
    return ewald.real_apply(x, q, L, xi), ewald.wave_apply(x, q, L, xi)


def _apply(h, x, q, parts):
    import torch
    out = torch.zeros((h.n, 11), dtype=torch.float64, device='cuda:0')
    h.mobility_apply(dev(x), dev(q), out, parts)
    return host(out)


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('precision', [0, 1])
def test_mobility_real_part(name, precision):
    from paper_1709_06946_amd import pse
    h, x, L = case(name, precision)
    ref, _ = oracle_parts(name)
    y = _apply(h, x, moments(name), pse.PSE_REAL)
    errs, perr = block_errors(y, ref), particle_errors(y, ref)
    print(name, precision, 'real', errs, perr)
    assert max(errs.values()) < TOL, errs
    assert max(perr.values()) < PARTICLE_TOL, perr


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('precision', [0, 1])
def test_mobility_wave_part(name, precision):
    from paper_1709_06946_amd import pse
    h, x, L = case(name, precision)
    _, ref = oracle_parts(name)
    y = _apply(h, x, moments(name), pse.PSE_WAVE)
    errs, perr = block_errors(y, ref), particle_errors(y, ref)
    print(name, precision, 'wave', errs, perr)
    assert max(errs.values()) < TOL, errs
    assert max(perr.values()) < PARTICLE_TOL, perr


@pytest.mark.parametrize('name', list(CASES))
def test_mobility_total(name):
    from paper_1709_06946_amd import pse
    h, x, L = case(name)
    r, w = oracle_parts(name)
    y = _apply(h, x, moments(name), pse.PSE_REAL | pse.PSE_WAVE)
    errs, perr = block_errors(y, r + w), particle_errors(y, r + w)
    print(name, 'total', errs, perr)
    assert max(errs.values()) < TOL, errs
    assert max(perr.values()) < PARTICLE_TOL, perr


def test_mobility_is_linear_and_symmetric():
    """<a, M b> = <M a, b> for the GPU operator (the grand mobility is
    symmetric in the stored coordinates)."""
    from paper_1709_06946_amd import pse
    h, x, L = case('phi0.1')
    rng = np.random.default_rng(5)
    a, b = rng.normal(size=(2, h.n, 11))
    Ma = _apply(h, x, a, pse.PSE_REAL | pse.PSE_WAVE)
    Mb = _apply(h, x, b, pse.PSE_REAL | pse.PSE_WAVE)
    assert abs((a * Mb).sum() - (Ma * b).sum()) < 1e-9 * abs((a * Mb).sum())
    M2a = _apply(h, x, 2.0 * a, pse.PSE_REAL | pse.PSE_WAVE)
    assert np.abs(M2a - 2.0 * Ma).max() < 1e-12 * np.abs(Ma).max()


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('precision', [0, 1])
def test_sampler_wave_same_noise(name, precision):
    import torch
    h, x, L = case(name, precision)
    g = h.derived.grid
    psi = inputs.wave_noise(g, CASES[name]['seed'] + 3)
    out = torch.zeros((h.n, 11), dtype=torch.float64, device='cuda:0')
    h.brownian_sample(dev(x), psi_wave=dev(psi), out_wave=out)
    ref = brownian.wave_sample(x, psi, L, g, h.derived.xi)
    errs, perr = block_errors(host(out), ref), particle_errors(host(out), ref)
    print(name, precision, 'wave sampler', errs, perr)
    assert max(errs.values()) < TOL, errs
    assert max(perr.values()) < PARTICLE_TOL, perr


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('precision', [0, 1])
def test_sampler_real_same_noise(name, precision):
    """Lanczos to 1e-8 (FP64) or 1e-5 (mixed: the FP32 pair sums bound the
    attainable change of the iterate near 1e-7)."""
    import torch
    h, x, L = case(name, precision, lanczos_tol=1e-8 if precision == 0 else 1e-5)
    psi = inputs.real_noise(h.n, CASES[name]['seed'] + 4)
    out = torch.zeros((h.n, 11), dtype=torch.float64, device='cuda:0')
    rc, st = h.brownian_sample(dev(x), psi_real=dev(psi), out_real=out)
    ref = brownian.real_sample(x, psi, L, h.derived.xi)
    errs, perr = block_errors(host(out), ref), particle_errors(host(out), ref)
    print(name, precision, 'real sampler', errs, perr, st)
    assert rc == 0 and st['converged'] == 1
    assert max(errs.values()) < TOL, errs
    assert max(perr.values()) < PARTICLE_TOL, perr


def test_sampler_real_default_tolerance():
    """At the Lanczos tolerance 1e-3 the iterate still matches the principal
    square root to the same order, in a handful of iterations."""
    import torch
    h, x, L = case('phi0.1')
    psi = inputs.real_noise(h.n, 99)
    out = torch.zeros((h.n, 11), dtype=torch.float64, device='cuda:0')
    rc, st = h.brownian_sample(dev(x), psi_real=dev(psi), out_real=out)
    ref = brownian.real_sample(x, psi, L, h.derived.xi)
    assert rel_err(host(out), ref) < 2e-3
    assert st['lanczos_iters'] <= 20


def test_philox_noise_statistics():
    """In-kernel Philox noise: the wave-space sample has the covariance of
    M_w over the grid (checked on the trace, per particle)."""
    import torch
    from paper_1709_06946_amd import pse
    h, x, L = case('phi0.1')
    out = torch.zeros((h.n, 11), dtype=torch.float64, device='cuda:0')
    acc = np.zeros((h.n, 11))
    nrep = 200
    for s in range(nrep):
        h.brownian_sample(dev(x), seed=1234, counter=s, out_wave=out)
        acc += host(out)**2
    var = acc / nrep
    Mw = brownian.wave_dense_grid(x, L, h.derived.grid, h.derived.xi)
    ref = np.diag(Mw).reshape(h.n, 11)
    ratio = var.sum() / ref.sum()
    assert abs(ratio - 1) < 0.03, ratio
    # same (seed, counter) reproduces the same draw
    h.brownian_sample(dev(x), seed=7, counter=3, out_wave=out)
    a = host(out)
    h.brownian_sample(dev(x), seed=7, counter=3, out_wave=out)
    assert np.array_equal(a, host(out))


@functools.lru_cache(maxsize=None)
def step_case(name, precision=0, with_noise=True):
    """One constrained step with given noise.  Krylov tolerances: 1e-8 for
    FP64; for the mixed form Lanczos 1e-5 and GMRES 1e-5 (FP32 inner solves
    inside the FP64 residual refinement, which must reach 1e-5 in FP64)."""
    import torch
    kt = 1e-8 if precision == 0 else 1e-5
    h, x, L = case(name, precision, lanczos_tol=kt, gmres_tol=kt)
    c = CASES[name]
    g = h.derived.grid
    FL = inputs.forces_torques(h.n, c['seed'] + 1)
    if with_noise:
        psi1 = inputs.real_noise(h.n, c['seed'] + 5)
        psi2 = inputs.wave_noise(g, c['seed'] + 6)
    else:
        psi1 = np.zeros((h.n, 11))
        psi2 = np.zeros((3, g, g, g // 2 + 1), complex)
    dt = 1e-3
    xt = dev(x)
    slip = torch.zeros((h.n, 11), dtype=torch.float64, device='cuda:0')
    S = torch.zeros((h.n, 5), dtype=torch.float64, device='cuda:0')
    U = torch.zeros((h.n, 3), dtype=torch.float64, device='cuda:0')
    rc, st = h.constrained_step(xt, dev(FL), dt, psi_real=dev(psi1), psi_wave=dev(psi2),
                                slip=slip, stresslet=S, velocity=U)
    gpu = dict(x1=host(xt), slip=host(slip), S=host(S), U=host(U), rc=rc, st=st)
    ref = integrator.midpoint_step(x, FL, psi1, psi2, dt, L, g, h.derived.xi,
                                   xi_total=7.0 / L)
    return gpu, ref, x, L, dt


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('precision', [0, 1])
def test_step_deterministic_constrained_velocity(name, precision):
    """Without noise the step velocity is the stresslet-constrained mobility
    applied to the forces and torques (Eq. constrained_vel)."""
    gpu, ref, x, L, dt = step_case(name, precision, with_noise=False)
    assert gpu['rc'] == 0 and gpu['st']['converged'] == 1
    eU, eS = rel_err(gpu['U'], ref['U']), rel_err(gpu['S'], ref['S'])
    pU, pS = particle_err(gpu['U'], ref['U']), particle_err(gpu['S'], ref['S'])
    print(name, precision, 'deterministic U', eU, pU, 'S', eS, pS, gpu['st'])
    assert eU < TOL and eS < TOL
    assert pU < PARTICLE_TOL and pS < PARTICLE_TOL
    if precision == 1:
        assert 0 <= gpu['st']['fp64_residual'] < 1e-5


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('precision', [0, 1])
def test_step_same_noise(name, precision):
    """The whole step with the same noise; for the mixed form this is the FP32
    GMRES inside the FP64 residual refinement against the FP64 oracle."""
    gpu, ref, x, L, dt = step_case(name, precision)
    assert gpu['rc'] == 0 and gpu['st']['converged'] == 1
    pairs = dict(slipU=(gpu['slip'][:, 0:3], ref['slip'][:, 0:3]),
                 slipE=(gpu['slip'][:, 6:11], ref['slip'][:, 6:11]),
                 S=(gpu['S'], ref['S']), U=(gpu['U'], ref['U']))
    dx = gpu['x1'] - x
    dx -= L * np.rint(dx / L)
    pairs['dx'] = (dx, ref['dx'])
    errs = {k: rel_err(*v) for k, v in pairs.items()}
    perr = {k: particle_err(*v) for k, v in pairs.items()}
    print(name, precision, 'step', errs, perr, gpu['st'])
    assert max(errs.values()) < TOL, errs
    assert max(perr.values()) < PARTICLE_TOL, perr
    if precision == 1:
        assert gpu['st']['refine_passes'] >= 1
        assert 0 <= gpu['st']['fp64_residual'] < 1e-5
    assert np.all((gpu['x1'] >= 0) & (gpu['x1'] < L))


@pytest.mark.parametrize('precision', [0, 1])
def test_graph_replays_match_eager_launches(precision):
    """Constrained steps with the operator replayed from captured graphs
    (default) and launched eagerly agree, over several steps in a row (each
    replay after the library's own eager work and synchronisations)."""
    import torch

    from paper_1709_06946_amd import pse
    c = CASES['phi0.1']
    x0, L = packing(c['N'], c['phi'], c['seed'])
    FL = np.random.default_rng(5).normal(size=(c['N'], 6))
    res = []
    for graphs in (0, -1):
        h = pse.PSE(c['N'], L, grid=c['grid'], tol=1e-3, precision=precision, graphs=graphs)
        x = dev(x0)
        stats = []
        for k in range(3):
            rc, st = h.constrained_step(x, dev(FL), 1e-3, seed=77, step=k)
            assert rc >= 0
            stats.append(st['gmres_iters'])
        res.append((host(x), stats))
        h.close()
    (xa, sa), (xb, sb) = res
    d = xa - xb
    d -= L * np.rint(d / L)
    disp = xa - x0
    disp -= L * np.rint(disp / L)
    assert sa == sb
    # every sum has a fixed order (cells and tiles ordered by particle index,
    # fixed reduction trees), so the replays reproduce the eager launches bit
    # for bit in both precisions
    assert np.array_equal(xa, xb), np.abs(d).max()
    assert np.abs(disp).max() > 0
