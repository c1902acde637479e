"""Pair mobility functions of the FTS (force-torque-stresslet) PSE kernel.

Oracle module (test infrastructure only).

The Fourier-space pair mobilities (Eqs. MUF, MUC, MDF, MDC) all have the form
shape factor x point-force kernel:

    M_UF  <->  (1/eta k^2) j0 j0 (I - kk)
    M_UC  <-> -(1/eta k^2) j0 (3i f1 k_n) (I - kk)
    M_DF  <->  (1/eta k^2) (3i f1 k_j) j0 (I - kk)
    M_DC  <-> -(1/eta k^2) (3i f1)^2 k_j k_n (I - kk)

with j0 = sin(ka)/ka and f1 = (sin ka - ka cos ka)/(ka)^3.  Writing
T_pq(r) for the inverse transform of f_p f_q (I - kk)/(eta k^2) (f_0 = j0,
f_1 = f1) and k_n <-> -i d/dr_n gives, for r = x_alpha - x_beta,

    M_UF_im   =        T00_im
    M_UC_imn  = -3 d_n T01_im
    M_DF_ijm  = +3 d_j T01_im
    M_DC_ijmn = -9 d_j d_n T11_im

and T_pq = (grad grad - I lap) phi_pq, where phi_pq is the inverse transform of
f_p f_q / (eta k^4).  For a radial phi(r) all derivatives follow from
Phi_n = ((1/r) d/dr)^n phi.  Only seven radial coefficient functions are
needed (the paper's F1,F2 / G1,G2 / K1,K2,K3 count, Appendix A):

    a  = -(r^2 Phi2 + 2 Phi1)   b  = r^2 Phi2        (pq = 00)
    c1 = r^3 Phi3               c2 = r Phi2          (pq = 01)
    d2 = Phi2   d3 = r^2 Phi3   d4 = r^4 Phi4        (pq = 11)

The splitting function H(k, xi) (Sec. II.B) divides each kernel into a
wave-space part (factor H) and a real-space part (factor 1 - H).  The
real-space part is evaluated here as  full - H-part:

* full: the free-space kernel.  f_0 and f_1 are the Fourier transforms of a
  uniform shell density delta(|x|-a)/(4 pi a^2) and of a uniform ball density
  1/(4 pi a^3), and 1/k^4 is the transform of -|x|/(8 pi).  So
  phi_pq = -(1/8 pi eta) (g_pq * |x|) with g_pq the convolution of the two
  densities, a radial polynomial density on |s| < 2a.  The spherical mean of
  |r - s n| is r + s^2/(3r) (s < r) and s + r^2/(3s) (s > r); the integrals
  are done exactly with sympy.
* H-part: Phi_n^H(r) = (1/(2 pi^2 eta)) int_0^inf H f_p f_q (-1)^n k^(2n-2)
  j_n(kr)/(kr)^n dk, using ((1/r) d/dr)^n j0(kr) = (-1)^n k^2n j_n(kr)/(kr)^n.
  The integrand decays like exp(-k^2/4 xi^2), so composite Gauss-Legendre on
  [0, 2 xi sqrt(50)] is exact to rounding.

Appendix A of the paper prints closed forms of the same real-space functions;
its UF functions agree with this module to rounding, the UC and DC ones do not
(readings listed in the design notes), which is why the oracle derives them.
"""
import functools

import numpy as np
import scipy.special as sps
import sympy as sp

COEFF_NAMES = ('a', 'b', 'c1', 'c2', 'd2', 'd3', 'd4')

# (pq, n) pairs of Phi_n^{pq} needed by the seven coefficient functions.
_PHI_NEEDED = (('00', 1), ('00', 2), ('01', 2), ('01', 3),
               ('11', 2), ('11', 3), ('11', 4))


@functools.lru_cache(maxsize=1)
def _full_coefficients_symbolic():
    """Exact free-space coefficient functions as lambdified (r, a) callables.

    Returns {name: (f_inside(r, a), f_outside(r, a))} for r < 2a and r >= 2a,
    without the common factor -1/(8 pi eta)."""
    r, s, a = sp.symbols('r s a', positive=True)
    # 4 pi s^2 g_pq(s): radial mass density of the convolution of the shape
    # densities (shell * shell, shell * ball, ball * ball), support s < 2a.
    # shell*shell: distance between two uniform points on the sphere has pdf
    #   s/(2a^2); shell*ball: fraction of a shell of radius a centred at s
    #   lying inside the ball is (2a - s)/(4a); ball*ball: lens volume
    #   pi (4a + s)(2a - s)^2 / 12.
    w = {
        '00': 4 * sp.pi * s**2 * (s / (2 * a**2)) / (4 * sp.pi * s**2),
        '01': 4 * sp.pi * s**2 * ((2 * a - s) / (4 * a)) / (4 * sp.pi * a**3),
        '11': 4 * sp.pi * s**2 * (sp.pi * (4 * a + s) * (2 * a - s)**2 / 12)
        / (4 * sp.pi * a**3)**2,
    }
    mean_out = r + s**2 / (3 * r)     # spherical mean of |r - s n|, s < r
    mean_in = s + r**2 / (3 * s)      # s > r
    phi = {}
    for pq, ws in w.items():
        inside = (sp.integrate(ws * mean_out, (s, 0, r))
                  + sp.integrate(ws * mean_in, (s, r, 2 * a)))
        outside = sp.integrate(ws * mean_out, (s, 0, 2 * a))
        phi[pq] = (sp.expand(inside), sp.expand(outside))

    def L(expr):                      # (1/r) d/dr
        return sp.expand(sp.diff(expr, r) / r)

    out = {}
    for region in (0, 1):
        P = {}
        for pq, n in _PHI_NEEDED:
            e = phi[pq][region]
            for _ in range(n):
                e = L(e)
            P[(pq, n)] = e
        co = {
            'a': -(r**2 * P[('00', 2)] + 2 * P[('00', 1)]),
            'b': r**2 * P[('00', 2)],
            'c1': r**3 * P[('01', 3)],
            'c2': r * P[('01', 2)],
            'd2': P[('11', 2)],
            'd3': r**2 * P[('11', 3)],
            'd4': r**4 * P[('11', 4)],
        }
        for name, e in co.items():
            out.setdefault(name, [None, None])[region] = sp.lambdify(
                (r, a), sp.expand(e), 'numpy')
    return out


def full_coefficients(r, a=1.0, eta=1.0):
    """Free-space coefficient functions {name: array} at separations r."""
    r = np.asarray(r, dtype=np.float64)
    sym = _full_coefficients_symbolic()
    pref = -1.0 / (8.0 * np.pi * eta)
    inside = r < 2.0 * a
    out = {}
    for name in COEFF_NAMES:
        fin, fout = sym[name]
        rin = np.where(inside, r, a)            # keep each branch finite
        rout = np.where(inside, 3.0 * a, r)
        vin = np.broadcast_to(fin(rin, a), r.shape)
        vout = np.broadcast_to(fout(rout, a), r.shape)
        out[name] = pref * np.where(inside, vin, vout)
    return out


def hasimoto_H(k, xi):
    """Splitting function H(k, xi) = (1 + k^2/4xi^2) exp(-k^2/4xi^2) (Sec. II.B)."""
    u = (np.asarray(k) / (2.0 * xi))**2
    return (1.0 + u) * np.exp(-u)


def jn_over_xn(n, x):
    """j_n(x)/x^n, accurate at small x (power series) and large x (scipy)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    small = x < 3.0
    xs = x[small]
    # sum_k (-x^2/2)^k / (k! (2n+2k+1)!!)
    term = np.full_like(xs, 1.0 / sps.factorial2(2 * n + 1, exact=True))
    acc = term.copy()
    t = -0.5 * xs * xs
    for k in range(1, 40):
        term = term * t / (k * (2 * n + 2 * k + 1))
        acc += term
    out[small] = acc
    xl = x[~small]
    out[~small] = sps.spherical_jn(n, xl) / xl**n
    return out


def shape_f(p, x):
    """Shape factors f_0 = sin x / x and f_1 = (sin x - x cos x)/x^3 (Eq. WSops)."""
    return jn_over_xn(p, x)


def _gauss_legendre_nodes(kmax, npanel, order=16):
    t, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(0.0, kmax, npanel + 1)
    h = np.diff(edges)
    mid = 0.5 * (edges[1:] + edges[:-1])
    k = (mid[:, None] + 0.5 * h[:, None] * t[None, :]).ravel()
    wk = (0.5 * h[:, None] * w[None, :]).ravel()
    return k, wk


def H_coefficients(r, xi, a=1.0, eta=1.0, u_max=50.0):
    """Coefficient functions of the H-filtered (wave-space, continuous) kernel.

    Phi_n^H(r) = 1/(2 pi^2 eta) int H f_p(ka) f_q(ka) (-1)^n k^(2n-2)
    j_n(kr)/(kr)^n dk, integrated to k = 2 xi sqrt(u_max) where
    H < 1e-19."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    kmax = 2.0 * xi * np.sqrt(u_max)
    rmax = float(r.max()) if r.size else 0.0
    npanel = max(16, int(np.ceil(kmax * (rmax + 2.0 * a + 1.0) / np.pi)))
    k, wk = _gauss_legendre_nodes(kmax, npanel)
    base = wk * hasimoto_H(k, xi) / (2.0 * np.pi**2 * eta)
    f = {0: shape_f(0, k * a), 1: shape_f(1, k * a)}
    weights = {}
    for pq, n in _PHI_NEEDED:
        p, q = int(pq[0]), int(pq[1])
        weights[(pq, n)] = base * f[p] * f[q] * (-1.0)**n * k**(2 * n - 2)
    Phi = {key: np.empty(r.shape) for key in weights}
    chunk = max(1, 2_000_000 // k.size)
    for s0 in range(0, r.size, chunk):
        rc = r[s0:s0 + chunk]
        X = np.outer(rc, k)
        J = {n: jn_over_xn(n, X) for n in (1, 2, 3, 4)}
        for (pq, n), wv in weights.items():
            Phi[(pq, n)][s0:s0 + chunk] = J[n] @ wv
    return {
        'a': -(r**2 * Phi[('00', 2)] + 2 * Phi[('00', 1)]),
        'b': r**2 * Phi[('00', 2)],
        'c1': r**3 * Phi[('01', 3)],
        'c2': r * Phi[('01', 2)],
        'd2': Phi[('11', 2)],
        'd3': r**2 * Phi[('11', 3)],
        'd4': r**4 * Phi[('11', 4)],
    }


def real_coefficients(r, xi, a=1.0, eta=1.0):
    """Real-space coefficient functions: full minus H-part (factor 1 - H)."""
    full = full_coefficients(r, a, eta)
    hp = H_coefficients(r, xi, a, eta)
    return {n: full[n] - hp[n] for n in COEFF_NAMES}


def cartesian_tensors(rhat, co):
    """Cartesian pair tensors (UF, UC, DF, DC) from unit vectors and coefficients.

    rhat: (M, 3); co: dict of (M,) arrays.  Terms carrying rhat vanish at
    r = 0 (their coefficients are zero there), so any rhat may be passed for
    the self term."""
    e = rhat
    d = np.eye(3)
    a, b = co['a'], co['b']
    c1, c2 = co['c1'], co['c2']
    d2, d3, d4 = co['d2'], co['d3'], co['d4']
    ee = np.einsum('Mi,Mj->Mij', e, e)
    UF = a[:, None, None] * d + b[:, None, None] * ee
    # dT01[i, m, n] = d_n T01_im
    eee = np.einsum('Mij,Mk->Mijk', ee, e)
    dT = (c1[:, None, None, None] * eee
          + c2[:, None, None, None] * (np.einsum('in,Mm->Mimn', d, e)
                                       + np.einsum('mn,Mi->Mimn', d, e))
          - (c1 + 4 * c2)[:, None, None, None] * np.einsum('im,Mn->Mimn', d, e))
    UC = -3.0 * dT                                   # [i, m, n]
    DF = 3.0 * np.transpose(dT, (0, 1, 3, 2))        # [i, j, m] = 3 d_j T_im
    # ddT[i, j, m, n] = d_j d_n T11_im
    eeee = np.einsum('Mij,Mmn->Mijmn', ee, ee)
    six = (np.einsum('ij,Mmn->Mijmn', d, ee) + np.einsum('im,Mjn->Mijmn', d, ee)
           + np.einsum('in,Mjm->Mijmn', d, ee) + np.einsum('jm,Min->Mijmn', d, ee)
           + np.einsum('jn,Mim->Mijmn', d, ee) + np.einsum('mn,Mij->Mijmn', d, ee))
    three = (np.einsum('ij,mn->ijmn', d, d) + np.einsum('im,jn->ijmn', d, d)
             + np.einsum('in,jm->ijmn', d, d))
    ddT = (d4[:, None, None, None, None] * eeee
           + d3[:, None, None, None, None] * six
           + d2[:, None, None, None, None] * three
           - np.einsum('im,Mjn->Mijmn', d,
                       (7 * d3 + d4)[:, None, None] * ee
                       + (5 * d2 + d3)[:, None, None] * d))
    DC = -9.0 * ddT
    return UF, UC, DF, DC
