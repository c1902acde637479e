"""Stresslet constraint and the mid-point SDAE step (oracle).

Test infrastructure only.

* Eq. rigidconstraint / constrained_vel: [U; 0] = M [F; S] gives
  S = -M_ES^{-1} M_EF F and U = (M_UF - M_US M_ES^{-1} M_EF) F.  M_ES is
  symmetric positive definite, so the dense solve is a Cholesky solve.
* Sec. III.D (four-step scheme) and Appendix B:
    1. slip (U^B, E^B) = sqrt(2 kT / dt) (M_r^(1/2) psi1 + M_w^(1/2) psi2)
       at x_k.  The sqrt(2kT/dt) factor is implied by the covariance stated
       in Appendix B and is applied here;
    2. x_{k+1/2} = x_k + dt/2 U^B;
    3. at x_{k+1/2}: [U; -E^B] = M [F^P; S] + [U^B; 0], i.e.
       M_ES S = -E^B - M_EF F^P and U = U^B + M_UF F^P + M_US S
       (the deterministic force/torque F^P enters the mid-point solve, a
       reading of Eq. eom combined with the four-step scheme);
    4. x_{k+1} = x_k + dt U.
  U here is the translational part; the generalized velocity (U, Omega) is
  also returned.
"""
import numpy as np

from . import brownian, ewald
from . import conventions as cv


def split_indices(N):
    iu = cv.block_indices(N, cv.IDX_UFRAK)     # (U, Omega) / (F, L)
    ie = cv.block_indices(N, cv.IDX_E)         # E / S
    return iu, ie


def constrained_solve(M, FL, rhs_extra=None):
    """Solve the stresslet constraint for a dense grand mobility M.

    FL: (N, 6) force and torque.  rhs_extra: optional (N, 5) added to the
    strain equation's right-hand side, i.e. M_ES S = -M_EF FL - rhs_extra.
    Returns (S (N,5), Ufrak (N,6) = M_UF FL + M_US S)."""
    N = M.shape[0] // 11
    iu, ie = split_indices(N)
    f = np.asarray(FL, np.float64).ravel()
    b = -(M[np.ix_(ie, iu)] @ f)
    if rhs_extra is not None:
        b = b - np.asarray(rhs_extra).ravel()
    C = np.linalg.cholesky(M[np.ix_(ie, ie)])
    S = np.linalg.solve(C.T, np.linalg.solve(C, b))
    Uf = M[np.ix_(iu, iu)] @ f + M[np.ix_(iu, ie)] @ S
    return S.reshape(N, 5), Uf.reshape(N, 6)


def constrained_mobility(M):
    """M_UF - M_US M_ES^{-1} M_EF (the inverse of R_FU)."""
    N = M.shape[0] // 11
    iu, ie = split_indices(N)
    return (M[np.ix_(iu, iu)]
            - M[np.ix_(iu, ie)] @ np.linalg.solve(M[np.ix_(ie, ie)],
                                                  M[np.ix_(ie, iu)]))


def wrap(x, L):
    return x - L * np.floor(x / L)


def midpoint_step(x0, FL, psi1, psi2, dt, L, Ng, xi, a=1.0, eta=1.0, kT=1.0,
                  xi_total=None):
    """One stresslet-constrained mid-point step.

    psi1: (N, 11) real noise; psi2: wave noise in the grid layout of
    brownian.py; Ng, xi: the grid and splitting used by the sampler (the
    wave noise lives on that grid).  xi_total: splitting used to build the
    full mobility at the mid-point (any value gives the same matrix).
    Returns a dict of every intermediate result."""
    x0 = np.asarray(x0, np.float64)
    N = x0.shape[0]
    y1 = brownian.real_sample(x0, psi1, L, xi, a, eta)
    y2 = brownian.wave_sample(x0, psi2, L, Ng, xi, a, eta)
    slip = np.sqrt(2.0 * kT / dt) * (y1 + y2)
    UB, EB = slip[:, cv.IDX_U], slip[:, cv.IDX_E]
    x_half = wrap(x0 + 0.5 * dt * UB, L)
    M = ewald.grand_dense(x_half, L, xi if xi_total is None else xi_total,
                          a, eta)
    S, Uf = constrained_solve(M, FL, rhs_extra=EB)
    U = UB + Uf[:, 0:3]
    dx = dt * U
    return dict(y_real=y1, y_wave=y2, slip=slip, x_half=x_half, S=S,
                U=U, Ufrak=Uf, dx=dx, x1=wrap(x0 + dx, L))


# ------------------------------------------------- RPY-level comparison --
#
# The unconstrained PSE of the performance comparison (Sec. IV): forces
# only, so the mobility reduces to its force-velocity block M_UF (the
# periodic RPY tensor as split by the positively split Ewald sum).  The
# split sampler restricted to that block gives the Brownian velocity
#   U^B = sqrt(2 kT / dt) ((M_r)_UF^(1/2) psi1 + (M_w)_UF^(1/2) psi2),
# with (M_r)_UF^(1/2) the principal root of the real-space UF block and the
# wave part the velocity rows of the wave sampler (whose covariance is the
# wave-space UF block).  M_UF is divergence-free, so an Euler-Maruyama step
#   x_{k+1} = x_k + dt (M_UF F + U^B)
# carries no drift term.

def rpy_mobility(x, L, xi, a=1.0, eta=1.0):
    """M_UF (3N x 3N): the force-velocity block of the full mobility."""
    N = np.asarray(x).shape[0]
    iu = cv.block_indices(N, cv.IDX_U)
    return ewald.grand_dense(x, L, xi, a, eta)[np.ix_(iu, iu)]


def rpy_step(x0, F, psi1, psi2, dt, L, Ng, xi, a=1.0, eta=1.0, kT=1.0, xi_total=None):
    """One unconstrained RPY-level step.

    F: (N, 3) or None; psi1: (N, 3) real noise; psi2: wave noise in the grid
    layout of brownian.py; Ng, xi: the sampler's grid and splitting.
    Returns a dict of every intermediate result."""
    x0 = np.asarray(x0, np.float64)
    N = x0.shape[0]
    iu = cv.block_indices(N, cv.IDX_U)
    Mr = ewald.real_dense(x0, L, xi, a, eta)[np.ix_(iu, iu)]
    y1 = brownian.principal_sqrt_apply(Mr, np.asarray(psi1, np.float64).ravel()).reshape(N, 3)
    y2 = brownian.wave_sample(x0, psi2, L, Ng, xi, a, eta)[:, cv.IDX_U]
    slip = np.sqrt(2.0 * kT / dt) * (y1 + y2)
    U = slip.copy()
    if F is not None:
        M = rpy_mobility(x0, L, xi if xi_total is None else xi_total, a, eta)
        U += (M @ np.asarray(F, np.float64).ravel()).reshape(N, 3)
    dx = dt * U
    return dict(y_real=y1, y_wave=y2, slip=slip, U=U, dx=dx, x1=wrap(x0 + dx, L))
