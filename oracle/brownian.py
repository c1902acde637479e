"""Split Brownian sampler (oracle), Sec. III "Fast Stochastic Sampling".

Test infrastructure only.

Eq. split: M^(1/2) dW is equal in distribution to M_r^(1/2) dW1 +
M_w^(1/2) dW2.  For same-noise comparisons both parts must be fixed
functions of the noise:

* real part: the principal square root of M_r (Sec. III.B, which the Lanczos
  iteration approximates), from a dense symmetric eigendecomposition;
* wave part: Eq. DFTsqrt, M_w^(1/2) dW2 = D^+ P^+ B^(1/2) dW2, written out as
  a direct non-uniform sum over exactly the grid's wave vectors:
      y_a = V^(-1/2) sum_k exp(i k.x_a) P(k)^+ sqrt(H/(eta k^2)) (I - kk) psi(k)
  with psi(-k) = conj(psi(k)) (the conjugacy condition).

Wave-noise layout (shared with the library interface): complex array
psi[c, iz, iy, ix], c = 0..2, shape (3, Ng, Ng, Ng//2 + 1); index i maps to
the integer wave number kappa = i for i < Ng/2 and i - Ng otherwise (ix is
kappa_x >= 0 directly).  Only the canonical half space is read:
kappa_x > 0, or kappa_x = 0 and kappa_y > 0, or kappa_x = kappa_y = 0 and
kappa_z > 0; every other entry is ignored and defined by conjugacy.  Modes
with any |kappa_i| = Ng/2 (Nyquist) and kappa = 0 carry no noise.  For a
covariance of M_w the real and imaginary parts of each canonical entry are
independent N(0, 1/2).
"""
import numpy as np

from . import ewald


def principal_sqrt_apply(M, v):
    """M^(1/2) v with the principal (symmetric PSD) square root."""
    lam, Q = np.linalg.eigh(M)
    lam = np.clip(lam, 0.0, None)
    return Q @ (np.sqrt(lam) * (Q.T @ v))


def grid_half_space(Ng, nmax=None):
    """Canonical half-space wave numbers of an Ng^3 grid, Nyquist excluded.

    nmax: if given, only wave numbers with |kappa| <= nmax (an optional
    truncation: the caller knows the terms beyond carry no weight or no
    noise).  Returns (kappa (K, 3) ints as (kx, ky, kz), array indices
    (K, 3) as (iz, iy, ix))."""
    h = Ng // 2
    lim = h - 1 if nmax is None else min(h - 1, int(np.floor(nmax)))
    g = np.arange(-lim, lim + 1)
    kx, ky, kz = np.meshgrid(g, g, g, indexing='ij')
    kap = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], -1)
    keep = ((kap[:, 0] > 0) | ((kap[:, 0] == 0) & (kap[:, 1] > 0))
            | ((kap[:, 0] == 0) & (kap[:, 1] == 0) & (kap[:, 2] > 0)))
    if nmax is not None:
        keep &= (kap**2).sum(1) <= nmax * nmax
    kap = kap[keep]
    idx = np.stack([kap[:, 2] % Ng, kap[:, 1] % Ng, kap[:, 0]], -1)
    return kap, idx


def wave_sample(x, psi, L, Ng, xi, a=1.0, eta=1.0, chunk=4096, kmax=None):
    """M_w^(1/2) psi over the Ng^3 grid's wave vectors; returns (N, 11).

    kmax: optional truncation of the sum to |k| <= kmax (for large grids:
    beyond kmax = 2 xi sqrt(50) the amplitude sqrt(H) is below e^-25)."""
    x = np.asarray(x, np.float64)
    V = L**3
    kap, idx = grid_half_space(Ng, None if kmax is None else kmax * L / (2 * np.pi))
    kvec = 2 * np.pi / L * kap
    ps = psi[:, idx[:, 0], idx[:, 1], idx[:, 2]].T           # (K, 3)
    out = np.zeros((x.shape[0], 11))
    for s0 in range(0, kvec.shape[0], chunk):
        kv = kvec[s0:s0 + chunk]
        PP = ewald.projected_shape(kv, a)                    # (I-kk)P, (K,3,11)
        amp = np.sqrt(ewald.wave_weight(kv, xi, eta) / V)
        vel = np.einsum('Kic,Ki->Kc', PP.conj(), amp[:, None] * ps[s0:s0 + chunk])
        ph = np.exp(1j * (kv @ x.T))                         # (K, N)
        out += 2.0 * np.real(np.einsum('Ka,Kc->ac', ph, vel))
    return out


def wave_dense_grid(x, L, Ng, xi, a=1.0, eta=1.0):
    """M_w restricted to the grid's wave vectors (the covariance of wave_sample)."""
    kap, _ = grid_half_space(Ng)
    return ewald.wave_dense(x, L, xi, a, eta, kvec=2 * np.pi / L * kap)


def real_sample(x, psi1, L, xi, a=1.0, eta=1.0):
    """M_r^(1/2) psi1 with psi1 of shape (N, 11); returns (N, 11)."""
    Mr = ewald.real_dense(x, L, xi, a, eta)
    return principal_sqrt_apply(Mr, np.asarray(psi1).ravel()).reshape(-1, 11)


def cholesky_sample(M, z):
    """Lower-Cholesky sample L z (valid in distribution only, Sec. III)."""
    return np.linalg.cholesky(M) @ z
