"""Quadrature parameter rules from the NUFFT error bound (oracle).

Test infrastructure only.

Eq. bound:  eps_q <= C [exp(-pi^2 P^2 / (2 m^2 lam)) + erfc(m / sqrt(2 lam))]
with lam the largest eigenvalue of A^T A for the lattice deformation A
(Eqs. lmax1, lmax2).  For an orthorhombic grid (lam = 1) the two terms are set
equal with erfc(x) <= exp(-x^2), which gives m = sqrt(pi P); then
2 exp(-pi P / 2) <= eps gives P = ceil((2/pi) ln(2/eps)).  Table 1 lists P
for deformed lattices; its rows are reproduced by keeping the orthorhombic
width m = sqrt(5 pi) (the eps = 1e-3 value) and requiring the first term to
be below eps/2: P = ceil(m sqrt(2 lam ln(2/eps)) / pi).
"""
import numpy as np


def lambda_max(A):
    """Largest eigenvalue of A^T A, from the definition."""
    A = np.asarray(A, np.float64)
    return float(np.linalg.eigvalsh(A.T @ A).max())


def shear_tensor(gamma):
    return np.array([[1.0, gamma, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def extension_tensor(e):
    return np.diag([e, 1.0 / e, 1.0])


def support_orthorhombic(eps):
    """P for lam = 1 with m = sqrt(pi P)."""
    return int(np.ceil(2.0 / np.pi * np.log(2.0 / eps)))


def support_deformed(eps, lam, m=np.sqrt(5.0 * np.pi)):
    """P for a deformed lattice at fixed Gaussian width m (Table 1 reading)."""
    return int(np.ceil(m * np.sqrt(2.0 * lam * np.log(2.0 / eps)) / np.pi))
