"""Dense real-space and wave-space parts of the periodic grand mobility (oracle).

Test infrastructure only.

Periodic box of side L, V = L^3, optionally deformed (Sec. II.C.2): with a
volume-preserving deformation A (det A = 1), the lattice vectors are the
columns of L A, the reciprocal vectors k = (2 pi / L) A^-T n (n integer) and
the real-space images x + L A n.  A = None is the cube.  All matrices are
11N x 11N in the stored coordinates of conventions.py, particle-major (row
11*alpha + c).

* Wave space (Eqs. MUFw-MDCw, WSops): for every reciprocal lattice vector
  k = 2 pi n / L, n != 0,
      M_w^{ab} = (1/V) sum_k exp(i k.(x_a - x_b)) P(k)^+ B'(k) P(k),
      B'(k) = H(k, xi) / (eta k^2) (I - kk),
      P(k) q = j0(ka) F - 3i f1(ka) C.k          (C from (L, s)),
  summed directly (no grid), truncated where H < 1e-19.  With
  A_a(k) = sqrt(w/V) exp(-i k.x_a) (I - kk) P(k) and k, -k paired,
  M_w = G^T G with G = sqrt(2) [Re A; Im A] over a half space of k, which is
  positive semi-definite by construction (Appendix C).
* Real space (Eqs. MUFr-MDCr, pairsums): image sum over the lattice of the
  real-space pair function of pairfuncs.py, truncated where
  exp(-xi^2 (r - 2a)^2) < 1e-18, including the self term r = 0.

M_w + M_r does not depend on xi (the split only moves terms between the two
sums); the tests check that, which pins both parts against each other.
"""
import numpy as np

from . import conventions as cv
from . import pairfuncs as pf

U_MAX = 50.0          # wave sum truncated at k^2/4xi^2 = U_MAX
R_TAIL = 6.5          # real sum truncated at r - 2a = R_TAIL / xi


# ----------------------------------------------------------------- k-space --

def _deformation(A):
    """(A, A^-1) with det A = 1 checked; identity for None."""
    if A is None:
        return np.eye(3), np.eye(3)
    A = np.asarray(A, np.float64)
    if abs(np.linalg.det(A) - 1.0) > 1e-12:
        raise ValueError('the lattice deformation must preserve volume (det A = 1)')
    return A, np.linalg.inv(A)


def wave_vectors(L, kmax, A=None):
    """Half-space reciprocal vectors k = (2 pi / L) A^-T n, n != 0, |k| <= kmax
    (n in the half space of half_space_lattice), as rows (K, 3)."""
    if A is None:
        return 2 * np.pi / L * half_space_lattice(L, kmax)
    A, Ai = _deformation(A)
    # |n| = |A^T k| L / 2 pi <= |A^T| kmax L / 2 pi
    nmax = int(np.floor(np.linalg.norm(A, 2) * kmax * L / (2 * np.pi))) + 1
    g = np.arange(-nmax, nmax + 1)
    n = np.stack(np.meshgrid(g, g, g, indexing='ij'), -1).reshape(-1, 3)
    keep = ((n[:, 0] > 0) | ((n[:, 0] == 0) & (n[:, 1] > 0))
            | ((n[:, 0] == 0) & (n[:, 1] == 0) & (n[:, 2] > 0)))
    k = 2 * np.pi / L * (n[keep] @ Ai)        # rows: (A^-T n)^T = n^T A^-1
    return k[(k**2).sum(1) <= kmax**2]


def half_space_lattice(L, kmax):
    """Integer vectors n != 0 with |2 pi n / L| <= kmax in one half space
    (n_x > 0, or n_x = 0 and n_y > 0, or n_x = n_y = 0 and n_z > 0)."""
    nmax = int(np.floor(kmax * L / (2 * np.pi)))
    g = np.arange(-nmax, nmax + 1)
    n = np.stack(np.meshgrid(g, g, g, indexing='ij'), -1).reshape(-1, 3)
    keep = ((n[:, 0] > 0) | ((n[:, 0] == 0) & (n[:, 1] > 0))
            | ((n[:, 0] == 0) & (n[:, 1] == 0) & (n[:, 2] > 0)))
    n = n[keep]
    k2 = (2 * np.pi / L)**2 * (n**2).sum(1)
    return n[k2 <= kmax**2]


def projected_shape(kvec, a):
    """(I - kk) P(k) for each k: complex array (K, 3, 11) (Eq. WSops)."""
    K = kvec.shape[0]
    k = np.sqrt((kvec**2).sum(1))
    khat = kvec / k[:, None]
    j0 = pf.shape_f(0, k * a)
    f1 = pf.shape_f(1, k * a)
    P = np.zeros((K, 3, 11), dtype=np.complex128)
    P[:, :, 0:3] = j0[:, None, None] * np.eye(3)
    # rho = -3i f1 C.k with C_mn = W[m, n, q] (L, s)_q
    P[:, :, 3:11] = -3j * f1[:, None, None] * np.einsum('mnq,Kn->Kmq', cv.W, kvec)
    proj = np.eye(3)[None] - np.einsum('Ki,Kj->Kij', khat, khat)
    return np.einsum('Kij,Kjc->Kic', proj, P)


def wave_weight(kvec, xi, eta):
    k2 = (kvec**2).sum(1)
    return pf.hasimoto_H(np.sqrt(k2), xi) / (eta * k2)


def wave_dense(x, L, xi, a=1.0, eta=1.0, kvec=None, chunk=2048, A=None):
    """Dense M_w (11N x 11N).  kvec: optional explicit half-space k set
    (default: every lattice vector of the (deformed) lattice up to the
    truncation)."""
    x = np.asarray(x, np.float64)
    N = x.shape[0]
    V = L**3
    if kvec is None:
        kvec = wave_vectors(L, 2 * xi * np.sqrt(U_MAX), A)
    M = np.zeros((11 * N, 11 * N))
    for s0 in range(0, kvec.shape[0], chunk):
        kv = kvec[s0:s0 + chunk]
        PP = projected_shape(kv, a)                            # (K,3,11)
        amp = np.sqrt(2.0 * wave_weight(kv, xi, eta) / V)
        ph = np.exp(-1j * (kv @ x.T))                          # (K,N)
        A = (amp[:, None, None, None] * ph[:, None, :, None]
             * PP[:, :, None, :])                              # (K,3,N,11)
        A = A.reshape(-1, 11 * N)
        Ar = np.ascontiguousarray(A.real)
        Ai = np.ascontiguousarray(A.imag)
        M += Ar.T @ Ar + Ai.T @ Ai
    return M


def wave_apply(x, q, L, xi, a=1.0, eta=1.0, kvec=None, chunk=4096, A=None):
    """Matrix-free M_w q for q of shape (N, 11) (direct k-sum)."""
    x = np.asarray(x, np.float64)
    q = np.asarray(q, np.float64)
    V = L**3
    if kvec is None:
        kvec = wave_vectors(L, 2 * xi * np.sqrt(U_MAX), A)
    out = np.zeros_like(q)
    for s0 in range(0, kvec.shape[0], chunk):
        kv = kvec[s0:s0 + chunk]
        PP = projected_shape(kv, a)                            # (K,3,11)
        w = wave_weight(kv, xi, eta) / V
        ph = np.exp(-1j * (kv @ x.T))                          # (K,N)
        rho = np.einsum('Kic,Kb,bc->Ki', PP, ph, q)            # (K,3)
        # out_a = sum over +-k = 2 Re[e^{ik.x_a} P^+ (I-kk) w rho]
        vel = np.einsum('Kic,Ki->Kc', PP.conj(), w[:, None] * rho)
        out += 2.0 * np.real(np.einsum('Ka,Kc->ac', ph.conj(), vel))
    return out


# -------------------------------------------------------------- real space --

def image_shifts(L, rcut, A=None):
    """Lattice vectors L A n (rows) covering every image within rcut of a
    separation already reduced to the cell around the origin."""
    if A is None:
        nimg = int(np.ceil(rcut / L)) + 1
        g = np.arange(-nimg, nimg + 1)
        return L * np.stack(np.meshgrid(g, g, g, indexing='ij'), -1).reshape(-1, 3)
    A, Ai = _deformation(A)
    # the cell's thinnest width is L / max_i |row i of A^-1|
    width = L / np.sqrt((Ai**2).sum(1)).max()
    nimg = int(np.ceil(rcut / width)) + 1
    g = np.arange(-nimg, nimg + 1)
    n = np.stack(np.meshgrid(g, g, g, indexing='ij'), -1).reshape(-1, 3)
    return L * n @ A.T


def reduce_image(d, L, A=None):
    """Separations (rows) reduced to the lattice cell around the origin: the
    lattice coordinates s = A^-1 d / L taken in [-1/2, 1/2)."""
    if A is None:
        return d - L * np.rint(d / L)
    A, Ai = _deformation(A)
    s = d @ Ai.T / L
    s -= np.rint(s)
    return L * s @ A.T


def image_pairs(x, L, rcut, A=None):
    """All (alpha, beta, separation) with |x_a - x_b + L A n| < rcut over the
    periodic lattice, alpha <= beta, including alpha == beta (n = 0 too)."""
    x = np.asarray(x, np.float64)
    N = x.shape[0]
    shifts = image_shifts(L, rcut, A)
    ia, ib = np.triu_indices(N)
    d = reduce_image(x[ia] - x[ib], L, A)
    out_a, out_b, out_r = [], [], []
    for sh in shifts:
        rr = d + sh
        dist = np.sqrt((rr**2).sum(1))
        m = dist < rcut
        out_a.append(ia[m])
        out_b.append(ib[m])
        out_r.append(rr[m])
    return (np.concatenate(out_a), np.concatenate(out_b), np.concatenate(out_r))


def pair_blocks(rvec, xi, a=1.0, eta=1.0, part='real'):
    """11x11 pair blocks M^{ab}(r) for separations r = x_a - x_b (M, 3).

    part: 'real' (factor 1 - H), 'full' (free space) or 'H' (factor H,
    continuous transform)."""
    rvec = np.atleast_2d(np.asarray(rvec, np.float64))
    r = np.sqrt((rvec**2).sum(1))
    rhat = np.where(r[:, None] > 0, rvec / np.where(r > 0, r, 1.0)[:, None],
                    np.array([1.0, 0.0, 0.0]))
    if part == 'real':
        co = pf.real_coefficients(r, xi, a, eta)
    elif part == 'full':
        co = pf.full_coefficients(r, a, eta)
    elif part == 'H':
        co = pf.H_coefficients(r, xi, a, eta)
    else:
        raise ValueError(part)
    return cv.cartesian_to_11(*pf.cartesian_tensors(rhat, co))


def real_cutoff(xi, a):
    return 2.0 * a + R_TAIL / xi


def real_dense(x, L, xi, a=1.0, eta=1.0, rcut=None, A=None):
    """Dense M_r (11N x 11N) by lattice image sum (Eq. pairsums)."""
    x = np.asarray(x, np.float64)
    N = x.shape[0]
    if rcut is None:
        rcut = real_cutoff(xi, a)
    ia, ib, rv = image_pairs(x, L, rcut, A)
    B = pair_blocks(rv, xi, a, eta, 'real')
    M = np.zeros((N, 11, N, 11))
    for p in range(ia.size):
        al, be = ia[p], ib[p]
        M[al, :, be, :] += B[p]
        if al != be:
            # M^{ba}(-r) = M^{ab}(r)^T
            M[be, :, al, :] += B[p].T
    return M.reshape(11 * N, 11 * N)


def real_apply(x, q, L, xi, a=1.0, eta=1.0, rcut=None, A=None):
    """Matrix-free M_r q for q of shape (N, 11)."""
    x = np.asarray(x, np.float64)
    q = np.asarray(q, np.float64)
    if rcut is None:
        rcut = real_cutoff(xi, a)
    ia, ib, rv = image_pairs(x, L, rcut, A)
    B = pair_blocks(rv, xi, a, eta, 'real')
    out = np.zeros_like(q)
    np.add.at(out, ia, np.einsum('pij,pj->pi', B, q[ib]))
    off = ia != ib
    np.add.at(out, ib[off], np.einsum('pji,pj->pi', B[off], q[ia[off]]))
    return out


def real_apply_rows(x, q, L, xi, rows, a=1.0, eta=1.0, rcut=None):
    """Rows `rows` of M_r q (Eq. pairsums for chosen output particles):
    out[alpha] = sum over partners beta and lattice vectors n with
    |x_alpha - x_beta + n L| < rcut of M^{alpha beta}(x_alpha - x_beta + n L) q_beta,
    the self block (beta = alpha, n = 0) included.  Each block is evaluated
    at its own separation (no transpose relation is used), so the cost is
    O(N) per row and full-size systems can be sampled."""
    x = np.asarray(x, np.float64)
    q = np.asarray(q, np.float64)
    if rcut is None:
        rcut = real_cutoff(xi, a)
    nimg = int(np.ceil(rcut / L)) + 1
    g = np.arange(-nimg, nimg + 1)
    shifts = L * np.stack(np.meshgrid(g, g, g, indexing='ij'), -1).reshape(-1, 3)
    out = np.zeros((len(rows), q.shape[1]))
    for k, al in enumerate(rows):
        d = x[al] - x
        d -= L * np.rint(d / L)
        rr = (d[:, None, :] + shifts[None, :, :]).reshape(-1, 3)
        beta = np.repeat(np.arange(x.shape[0]), shifts.shape[0])
        m = np.sqrt((rr**2).sum(1)) < rcut
        B = pair_blocks(rr[m], xi, a, eta, 'real')
        out[k] = np.einsum('pij,pj->i', B, q[beta[m]])
    return out


def grand_dense(x, L, xi, a=1.0, eta=1.0, A=None):
    """Full grand mobility M = M_w + M_r (independent of xi)."""
    return wave_dense(x, L, xi, a, eta, A=A) + real_dense(x, L, xi, a, eta, A=A)
