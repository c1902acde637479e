"""Closed-form real-space scalar mobility functions printed in the paper.

Fixture transcribed from Appendix A ("Real Space Scalar Mobility Functions")
of Fiore & Swan, arXiv 1709.06946.  Only the functions that are consistent
with the paper's own Fourier definitions (Eqs. MUF-MDC with the splitting
H(k, xi)) are transcribed:

* F1, F2 (velocity-force, cases r > 2a and r <= 2a) and the UF self term;
* G2 (velocity-couplet, both cases) and G1 for r > 2a;
* K3 (velocity gradient-couplet, both cases) and the DC self value K1(0)
  (valid at a = 1, where its powers of a do not matter).

Every function is  X(r) = x0 + x1 e^{-r^2 xi^2} + x2 e^{-(r-2a)^2 xi^2}
+ x3 e^{-(r+2a)^2 xi^2} + x4 erfc(r xi) + x5 erfc((r-2a) xi)
+ x6 erfc((r+2a) xi), with x0 = 0 for r > 2a.
"""
import numpy as np
from scipy.special import erfc

SQPI = np.sqrt(np.pi)


def _combo(c, r, xi, a):
    return (c[0] + c[1] * np.exp(-r * r * xi * xi)
            + c[2] * np.exp(-(r - 2 * a)**2 * xi * xi)
            + c[3] * np.exp(-(r + 2 * a)**2 * xi * xi)
            + c[4] * erfc(r * xi) + c[5] * erfc((r - 2 * a) * xi)
            + c[6] * erfc((r + 2 * a) * xi))


def F1(r, xi, a=1.0):
    """6 pi eta a M_UF = F1 (I - rr) + F2 rr (Appendix A, M_UF)."""
    f1 = (18 * r**2 * xi**2 + 3) / (64 * SQPI * a * r**2 * xi**3)
    f2 = ((2 * xi**2 * (2 * a - r) * (4 * a**2 + 4 * a * r + 9 * r**2)
           - 2 * a - 3 * r) / (128 * SQPI * a * r**3 * xi**3))
    f3 = ((-2 * xi**2 * (2 * a + r) * (4 * a**2 - 4 * a * r + 9 * r**2)
           + 2 * a - 3 * r) / (128 * SQPI * a * r**3 * xi**3))
    f4 = (3 - 36 * r**4 * xi**4) / (128 * a * r**3 * xi**4)
    f5 = ((4 * xi**4 * (r - 2 * a)**2 * (4 * a**2 + 4 * a * r + 9 * r**2) - 3)
          / (256 * a * r**3 * xi**4))
    f6 = ((4 * xi**4 * (2 * a + r)**2 * (4 * a**2 - 4 * a * r + 9 * r**2) - 3)
          / (256 * a * r**3 * xi**4))
    f0 = np.where(r > 2 * a, 0.0,
                  -(r - 2 * a)**2 * (4 * a**2 + 4 * a * r + 9 * r**2)
                  / (32 * a * r**3))
    return _combo([f0, f1, f2, f3, f4, f5, f6], r, xi, a)


def F2(r, xi, a=1.0):
    f1 = (6 * r**2 * xi**2 - 3) / (32 * SQPI * a * r**2 * xi**3)
    f2 = ((-2 * xi**2 * (r - 2 * a)**2 * (2 * a + 3 * r) + 2 * a + 3 * r)
          / (64 * SQPI * a * r**3 * xi**3))
    f3 = ((2 * xi**2 * (2 * a + r)**2 * (2 * a - 3 * r) - 2 * a + 3 * r)
          / (64 * SQPI * a * r**3 * xi**3))
    f4 = -3 * (4 * r**4 * xi**4 + 1) / (64 * a * r**3 * xi**4)
    f5 = ((3 - 4 * xi**4 * (2 * a - r)**3 * (2 * a + 3 * r))
          / (128 * a * r**3 * xi**4))
    f6 = ((3 - 4 * xi**4 * (2 * a - 3 * r) * (2 * a + r)**3)
          / (128 * a * r**3 * xi**4))
    f0 = np.where(r > 2 * a, 0.0,
                  (2 * a - r)**3 * (2 * a + 3 * r) / (16 * a * r**3))
    return _combo([f0, f1, f2, f3, f4, f5, f6], r, xi, a)


def uf_self(xi, a=1.0):
    """6 pi eta a M_UF^{aa,(r)} / delta (Appendix A, M_UF case 3)."""
    return ((1 - np.exp(-4 * a**2 * xi**2) + 4 * SQPI * a * xi * erfc(2 * a * xi))
            / (4 * SQPI * xi * a))


def G1_far(r, xi, a=1.0):
    """G1 for r > 2a (Appendix A, M_UC case 1)."""
    g1 = (-30 * r**4 * xi**4 + 15 * r**2 * xi**2 + 9) / (64 * SQPI * a**4 * r**3 * xi**5)
    g2 = ((3 * xi**2 * (2 * a - r) * (8 * a**2 + 16 * a * r + 25 * r**2)
           - 6 * xi**4 * (2 * a - r) * (32 * a**4 + 32 * a**3 * r + 44 * a**2 * r**2
                                        + 36 * a * r**3 + 25 * r**4)
           - 9 * (2 * a + 5 * r)) / (640 * SQPI * a**4 * r**4 * xi**5))
    g3 = ((-3 * xi**2 * (2 * a + r) * (8 * a**2 - 16 * a * r + 25 * r**2)
           + 6 * xi**4 * (2 * a + r) * (32 * a**4 - 32 * a**3 * r + 44 * a**2 * r**2
                                        - 36 * a * r**3 + 25 * r**4)
           + 18 * a - 45 * r) / (640 * SQPI * a**4 * r**4 * xi**5))
    g4 = (60 * r**6 * xi**6 + 9 * r**2 * xi**2 + 9) / (128 * a**4 * r**4 * xi**6)
    g5 = -3 * (512 * a**6 * xi**6 + 5 * r**2 * xi**2 * (64 * a**4 * xi**4 + 3)
               - 256 * a * r**5 * xi**6 + 100 * r**6 * xi**6 + 15) / (1280 * a**4 * r**4 * xi**6)
    g6 = -3 * (512 * a**6 * xi**6 + 5 * r**2 * xi**2 * (64 * a**4 * xi**4 + 3)
               + 256 * a * r**5 * xi**6 + 100 * r**6 * xi**6 + 15) / (1280 * a**4 * r**4 * xi**6)
    return _combo([0.0, g1, g2, g3, g4, g5, g6], r, xi, a)


def G2(r, xi, a=1.0):
    """G2 (Appendix A, M_UC, both cases)."""
    P = 16 * a**3 + 24 * a**2 * r + 14 * a * r**2 + 5 * r**3
    Q = 16 * a**3 - 24 * a**2 * r + 14 * a * r**2 - 5 * r**3
    g1 = (-6 * r**4 * xi**4 + 3 * r**2 * xi**2 - 9) / (64 * SQPI * a**4 * r**3 * xi**5)
    g2 = ((6 * xi**4 * (r - 2 * a)**2 * P - 3 * xi**2 * P + 18 * a + 45 * r)
          / (640 * SQPI * a**4 * r**4 * xi**5))
    g3 = ((-6 * xi**4 * (2 * a + r)**2 * Q + 3 * xi**2 * Q - 18 * a + 45 * r)
          / (640 * SQPI * a**4 * r**4 * xi**5))
    g4 = (12 * r**6 * xi**6 + 9 * r**2 * xi**2 - 9) / (128 * a**4 * r**4 * xi**6)
    g5 = ((12 * xi**6 * (128 * a**6 - 80 * a**4 * r**2 + 16 * a * r**5 - 5 * r**6)
           - 45 * r**2 * xi**2 + 45) / (1280 * a**4 * r**4 * xi**6))
    g6 = ((12 * xi**6 * (128 * a**6 - 80 * a**4 * r**2 - 16 * a * r**5 - 5 * r**6)
           - 45 * r**2 * xi**2 + 45) / (1280 * a**4 * r**4 * xi**6))
    g0 = np.where(r > 2 * a, 0.0,
                  -3 * (128 * a**6 - 80 * a**4 * r**2 + 16 * a * r**5 - 5 * r**6)
                  / (160 * a**4 * r**4))
    return _combo([g0, g1, g2, g3, g4, g5, g6], r, xi, a)


def K3(r, xi, a=1.0):
    """K3 (Appendix A, M_DC, both cases)."""
    k1 = (9 * (32 * a**2 * xi**2 * (-2 * r**4 * xi**4 + r**2 * xi**2 + 15)
               + 8 * r**6 * xi**6 - 4 * r**4 * xi**4 + 18 * r**2 * xi**2 - 45)
          / (4096 * SQPI * a**6 * r**4 * xi**7))
    k2 = (9 * (-8 * xi**6 * (r - 2 * a)**2 * (2 * a + r)**3 * (4 * a**2 + r**2)
               + 4 * xi**4 * (2 * a + r)**3 * (4 * a**2 + r**2)
               - 6 * xi**2 * (2 * a + r)**2 * (2 * a + 3 * r) + 45 * (r - 2 * a))
          / (8192 * SQPI * a**6 * r**5 * xi**7))
    k3 = (9 * (-8 * xi**6 * (r - 2 * a)**3 * (2 * a + r)**2 * (4 * a**2 + r**2)
               + 4 * xi**4 * (r - 2 * a)**3 * (4 * a**2 + r**2)
               + 6 * xi**2 * (r - 2 * a)**2 * (2 * a - 3 * r) + 45 * (2 * a + r))
          / (8192 * SQPI * a**6 * r**5 * xi**7))
    k4 = (9 * (8 * xi**2 * (4 * a**2 * (4 * r**6 * xi**6 - 9 * r**2 * xi**2 + 15)
                            - 2 * r**8 * xi**6 - 3 * r**4 * xi**2 + 6 * r**2) - 45)
          / (8192 * a**6 * r**5 * xi**8))
    k5 = (9 * (16 * xi**8 * (r**2 - 4 * a**2)**3 * (4 * a**2 + r**2)
               + 24 * r**2 * xi**4 * (12 * a**2 + r**2)
               - 48 * xi**2 * (10 * a**2 + r**2) + 45)
          / (16384 * a**6 * r**5 * xi**8))
    k0 = np.where(r > 2 * a, 0.0,
                  9 * (4 * a**2 - r**2)**3 * (4 * a**2 + r**2) / (512 * a**6 * r**5))
    return _combo([k0, k1, k2, k3, k4, k5, k5], r, xi, a)


def dc_self_K1(xi, a=1.0):
    """K1(0): 6 pi eta a M_DC^{aa,(r)} = K1(0) (basis tensor) at a = 1
    (Appendix A, M_DC case 3)."""
    return (-3 * (6 * a**2 * xi**2 + 1) / (80 * SQPI * a**6 * xi**3)
            + 3 * (10 * a**2 * xi**2 + 1) / (80 * SQPI * a**6 * xi**3)
            * np.exp(-4 * a**2 * xi**2)
            - 3 / (10 * a**3) * erfc(2 * a * xi))
