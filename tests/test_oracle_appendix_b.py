"""Pins of the oracle's mid-point step against Appendix B (weak accuracy).

Appendix B fixes the first two moments of one step of the four-step scheme
with the slip (U^B, E^B) drawn with covariance (2 kT / dt) M:

    <dx>     = kT dt  div R_FU^{-1} + O(dt^2)
    <dx dx>  = 2 kT dt R_FU^{-1}    + O(dt^2),
    R_FU^{-1} = M_UF - M_US M_ES^{-1} M_EF.

The oracle's step is a function of its noise through the unscaled slip
y = M_r^(1/2) psi1 + M_w^(1/2) psi2, which is N(0, M_r + M_w) when the noise
is standard (the split sampler, pinned in test_oracle_pins.py).  Setting
psi1 = M_r^(-1/2) v with the principal root gives y = v exactly, so the
step's response to every slip direction is probed one at a time:

* the linear response G (dx = G y + O(|y|^2)) by central differences, then
  Cov(dx) = G (M_r + M_w) G^T;
* the quadratic response along each eigenvector u_j of M_r + M_w (the even
  part of dx(s u_j), Richardson-extrapolated in s), whose eigenvalue-weighted
  sum is the exact O(dt) mean of dx.

Both are compared with the right-hand sides above, built from the dense
mobility (div R_FU^{-1} by central differences in the positions).  The
sampler's wave vectors are those of the Ng^3 grid; xi is small enough that
the Hasimoto factor beyond them is ~1e-11, so the sampled covariance and the
solve's full-lattice mobility agree to that level.
"""
import numpy as np
import pytest

from oracle import brownian, ewald, integrator

L, NG, XI, DT, KT = 7.0, 8, 0.34, 1e-3, 1.0
X0 = np.array([[1.0, 1.0, 1.0], [2.9, 1.6, 1.3]])     # near contact (r = 2.02a)
N = X0.shape[0]


def _sampler_cov():
    return ewald.real_dense(X0, L, XI) + brownian.wave_dense_grid(X0, L, NG, XI)


def _steering():
    """psi1 = R^{-1} v maps the slip v to real-space noise (R = M_r^(1/2))."""
    lam, Q = np.linalg.eigh(ewald.real_dense(X0, L, XI))
    assert lam.min() > 1e-6 * lam.max()
    return Q @ np.diag(1.0 / np.sqrt(lam)) @ Q.T


ZERO_WAVE = np.zeros((3, NG, NG, NG // 2 + 1), complex)


def _dx(step, Rinv, v, psi2=ZERO_WAVE):
    psi1 = (Rinv @ v).reshape(N, 11)
    out = step(X0, np.zeros((N, 6)), psi1, psi2, DT, L, NG, XI, kT=KT)
    return out['dx'].ravel()


IU = np.array([6 * p + i for p in range(N) for i in range(3)])


def _constrained(M):
    """Translational block of M_UF - M_US M_ES^-1 M_EF (the torque-free
    spheres' rotation is not part of the positions)."""
    return integrator.constrained_mobility(M)[np.ix_(IU, IU)]


def _appendix_b_cov():
    return 2.0 * KT * DT * _constrained(ewald.grand_dense(X0, L, XI))


def _appendix_b_mean():
    """kT dt div R_FU^{-1}: (div Mc)_{ai} = sum_{b,l} d Mc_{ai,bl} / d x_{bl},
    central differences with one Richardson step."""
    def dcol(b, l, d):
        xp, xm = X0.copy(), X0.copy()
        xp[b, l] += d
        xm[b, l] -= d
        Mp = _constrained(ewald.grand_dense(xp, L, XI))
        Mm = _constrained(ewald.grand_dense(xm, L, XI))
        return (Mp[:, 3 * b + l] - Mm[:, 3 * b + l]) / (2 * d)
    div = np.zeros(3 * N)
    for b in range(N):
        for l in range(3):
            d = 2e-3
            div += (4 * dcol(b, l, d) - dcol(b, l, 2 * d)) / 3
    return KT * DT * div


def _step_cov(step, Rinv, Mg):
    s = 1e-4
    G = np.zeros((3 * N, 11 * N))
    for j in range(11 * N):
        e = np.zeros(11 * N)
        e[j] = s
        G[:, j] = (_dx(step, Rinv, e) - _dx(step, Rinv, -e)) / (2 * s)
    return G @ Mg @ G.T


def _step_mean(step, Rinv, Mg):
    lam, U = np.linalg.eigh(Mg)
    mean = np.zeros(3 * N)
    for j in range(11 * N):
        u = U[:, j]
        q = []
        for s in (0.05, 0.1):
            q.append((_dx(step, Rinv, s * u) + _dx(step, Rinv, -s * u)) / (2 * s * s))
        mean += lam[j] * (4 * q[0] - q[1]) / 3
    return mean


@pytest.fixture(scope='module')
def fixed():
    return _steering(), _sampler_cov()


def test_wave_noise_enters_through_the_same_slip(fixed):
    """The wave-space noise moves the particles exactly as real-space noise
    producing the same slip does (so probing the slip with psi1 alone covers
    the wave noise too)."""
    Rinv, _ = fixed
    rng = np.random.default_rng(7)
    psi2 = (rng.normal(size=ZERO_WAVE.shape) + 1j * rng.normal(size=ZERO_WAVE.shape)) * 0.5
    y2 = brownian.wave_sample(X0, psi2, L, NG, XI).ravel()
    a = _dx(integrator.midpoint_step, Rinv, np.zeros(11 * N), psi2)
    b = _dx(integrator.midpoint_step, Rinv, y2)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_step_covariance_is_2kTdt_constrained_mobility(fixed):
    """Appendix B: <dx dx> = 2 kT dt (M_UF - M_US M_ES^-1 M_EF) (O(dt^2) terms
    vanish in the linear response)."""
    Rinv, Mg = fixed
    cov = _step_cov(integrator.midpoint_step, Rinv, Mg)
    ref = _appendix_b_cov()
    assert np.abs(cov - ref).max() <= 1e-11 * np.abs(ref).max()
    # the noise prefactor is pinned: half the variance is far outside
    half = _step_cov(lambda *a, **k: integrator.midpoint_step(*a, **{**k, 'kT': KT / 2}),
                     Rinv, Mg)
    assert np.abs(half - ref).max() > 0.4 * np.abs(ref).max()


def test_step_mean_is_kTdt_divergence_of_constrained_mobility(fixed):
    """Appendix B: <dx> = kT dt div R_FU^{-1} + O(dt^2) (the thermal drift
    comes from evaluating the constraint at the half-step point)."""
    Rinv, Mg = fixed
    mean = _step_mean(integrator.midpoint_step, Rinv, Mg)
    ref = _appendix_b_mean()
    assert np.abs(ref).max() > 1e-4 * DT * KT         # a drift to pin
    assert np.abs(mean - ref).max() <= 1e-7 * np.abs(ref).max()


def test_full_step_to_the_midpoint_fails_the_mean_pin(fixed, monkeypatch):
    """A planted mistake in the oracle (the constraint solved at
    x_k + dt U^B instead of x_k + dt/2 U^B) doubles the drift and is caught."""
    Rinv, Mg = fixed
    real_grand = ewald.grand_dense

    def moved(x, *a, **k):
        d = x - X0
        d -= L * np.rint(d / L)
        return real_grand(X0 + 2 * d, *a, **k)

    monkeypatch.setattr(integrator.ewald, 'grand_dense', moved)
    mean = _step_mean(integrator.midpoint_step, Rinv, Mg)
    monkeypatch.undo()
    ref = _appendix_b_mean()
    assert np.abs(mean - 2 * ref).max() <= 1e-5 * np.abs(ref).max()


def test_rpy_step_covariance_is_2kTdt_uf_mobility():
    """The RPY-level comparison step (Euler-Maruyama with the split sampler
    on the force-velocity block): its displacement is linear in the noise,
    with covariance 2 kT dt M_UF and zero mean (M_UF is divergence-free, so
    there is no drift).  Probed like the constrained step, steering the
    real-space noise through the principal root of the real UF block."""
    from oracle import conventions as cv
    iu = cv.block_indices(N, cv.IDX_U)
    Mr = ewald.real_dense(X0, L, XI)[np.ix_(iu, iu)]
    Mg = Mr + brownian.wave_dense_grid(X0, L, NG, XI)[np.ix_(iu, iu)]
    lam, Q = np.linalg.eigh(Mr)
    Rinv = Q @ np.diag(1.0 / np.sqrt(lam)) @ Q.T
    G = np.zeros((3 * N, 3 * N))
    for j in range(3 * N):
        e = np.zeros(3 * N)
        e[j] = 1.0
        G[:, j] = integrator.rpy_step(X0, None, (Rinv @ e).reshape(N, 3), ZERO_WAVE, DT, L, NG,
                                      XI, kT=KT)['dx'].ravel()
    ref = 2.0 * KT * DT * ewald.grand_dense(X0, L, XI)[np.ix_(iu, iu)]
    assert np.abs(G @ Mg @ G.T - ref).max() <= 1e-11 * np.abs(ref).max()
    # the wave noise enters through the same slip
    rng = np.random.default_rng(8)
    psi2 = (rng.normal(size=ZERO_WAVE.shape) + 1j * rng.normal(size=ZERO_WAVE.shape)) * 0.5
    y2 = brownian.wave_sample(X0, psi2, L, NG, XI)[:, cv.IDX_U].ravel()
    a = integrator.rpy_step(X0, None, np.zeros((N, 3)), psi2, DT, L, NG, XI, kT=KT)['dx']
    b = integrator.rpy_step(X0, None, (Rinv @ y2).reshape(N, 3), ZERO_WAVE, DT, L, NG, XI,
                            kT=KT)['dx']
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    # zero mean: the noise-free step does not move the particles
    z = integrator.rpy_step(X0, None, np.zeros((N, 3)), ZERO_WAVE, DT, L, NG, XI, kT=KT)['dx']
    assert np.abs(z).max() == 0.0
