"""The constraint solve's right preconditioner, checked on the oracle's dense
M_ES (N = 100, phi = 0.1): P = (1 + d/a0)/a0 - M_r,ES/a0^2, with d the
real-space self term and a0 = 3/(20 pi eta a^3), reduces the GMRES
iterations to 1e-4, and S = P y solves M_ES S = b to the same tolerance (the
residual that right-preconditioned GMRES minimises is the system's own).
A preconditioner with the wrong sign of the pair part, or a0 off by a
factor, loses the gain.  Host only: plain numpy GMRES on the oracle."""
import numpy as np
import pytest

from oracle import ewald
from paper_1709_06946_amd import inputs


def _gmres(A, b, tol, P=None, maxit=60):
    beta = np.linalg.norm(b)
    n = len(b)
    V = np.zeros((n, maxit + 1))
    H = np.zeros((maxit + 1, maxit))
    V[:, 0] = b / beta
    for j in range(maxit):
        w = A @ (P @ V[:, j] if P is not None else V[:, j])
        for _ in range(2):
            h = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ h
            H[:j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / H[j + 1, j]
        e1 = np.zeros(j + 2)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)
        if np.linalg.norm(H[:j + 2, :j + 1] @ y - e1) / beta < tol:
            x = V[:, :j + 1] @ y
            return j + 1, (P @ x if P is not None else x)
    raise AssertionError('no convergence')


@pytest.fixture(scope='module')
def system():
    N = 100
    x, L = inputs.packing(N, 0.1, seed=inputs.SEED_BASE + 61)
    xi = 0.6
    es = np.concatenate([np.arange(p * 11 + 6, p * 11 + 11) for p in range(N)])
    Mr = ewald.real_dense(x, L, xi)[np.ix_(es, es)]
    Mw = ewald.wave_dense(x, L, xi)[np.ix_(es, es)]
    return Mr, Mr + Mw


def _precond(Mr, a0, sign=1.0):
    d = np.mean(np.diag(Mr))
    n = len(Mr)
    return (1.0 + d / a0) / a0 * np.eye(n) - sign * Mr / a0**2


def test_preconditioner_reduces_iterations_and_keeps_the_solution(system):
    Mr, A = system
    a0 = 3.0 / (20.0 * np.pi)
    # the whole operator's diagonal is the isolated sphere's self term
    assert abs(np.mean(np.diag(A)) / a0 - 1.0) < 1e-3
    rng = np.random.default_rng(7)
    P = _precond(Mr, a0)
    for _ in range(3):
        b = rng.normal(size=len(A))
        k0, S0 = _gmres(A, b, 1e-4)
        k1, S1 = _gmres(A, b, 1e-4, P)
        assert k1 < k0, (k0, k1)
        assert np.linalg.norm(A @ S1 - b) / np.linalg.norm(b) < 1e-4
        assert np.linalg.norm(S1 - S0) / np.linalg.norm(S0) < 1e-3


def test_wrong_preconditioners_lose_the_gain(system):
    Mr, A = system
    a0 = 3.0 / (20.0 * np.pi)
    b = np.random.default_rng(8).normal(size=len(A))
    k = _gmres(A, b, 1e-4, _precond(Mr, a0))[0]
    assert _gmres(A, b, 1e-4, _precond(Mr, a0, sign=-1.0))[0] > k
    assert _gmres(A, b, 1e-4, _precond(Mr, 10.0 * a0))[0] > k
