"""Component layout of the generalized force and velocity (oracle).

Sec. II.B ("Mobility relation for rigid particles") splits the couplet C into
the torque L (antisymmetric part) and the stresslet S (symmetric part), and the
velocity gradient D into the angular velocity Omega and the rate of strain E.
The paper leaves the storage basis and the sign of the epsilon contractions
open; this module fixes them (readings listed in the design notes):

* Couplet index order follows the mobility formulas (Eqs. UC, DC): C_mn has the
  force component first and the surface-normal component second, and
  D_ij = d u_i / d x_j (Eq. fax2a).
* L = integral of y x f and Omega = curl(u)/2, which gives
  C^A_mn = -1/2 eps_mnk L_k and D^A_ij = -eps_ijk Omega_k, so that the power
  pairs as F.U + L.Omega + S:E.
* S and E are stored in an orthonormal (Frobenius) basis Y_1..Y_5 of
  symmetric traceless tensors, so that the 11N x 11N grand mobility is a
  symmetric matrix in the stored coordinates.

Per particle the generalized force is [F_x F_y F_z | L_x L_y L_z | s_1..s_5]
and the generalized velocity is [U | Omega | e_1..e_5].
"""
import numpy as np

NCOMP = 11

_R2 = 1.0 / np.sqrt(2.0)
_R6 = 1.0 / np.sqrt(6.0)

# Orthonormal symmetric traceless basis: Y_q : Y_p = delta_qp.
Y = np.zeros((5, 3, 3))
Y[0, 0, 1] = Y[0, 1, 0] = _R2            # (xy + yx)/sqrt2
Y[1, 0, 2] = Y[1, 2, 0] = _R2            # (xz + zx)/sqrt2
Y[2, 1, 2] = Y[2, 2, 1] = _R2            # (yz + zy)/sqrt2
Y[3, 0, 0], Y[3, 1, 1] = _R2, -_R2       # (xx - yy)/sqrt2
Y[4, 0, 0] = Y[4, 1, 1] = _R6            # (xx + yy - 2zz)/sqrt6
Y[4, 2, 2] = -2.0 * _R6

EPS = np.zeros((3, 3, 3))
for (i, j, k), sgn in {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1,
                       (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}.items():
    EPS[i, j, k] = sgn

# W[m, n, q]: couplet C_mn produced by the q-th entry of (L_1..L_3, s_1..s_5).
W = np.zeros((3, 3, 8))
W[:, :, 0:3] = -0.5 * EPS                 # C^A_mn = -1/2 eps_mnk L_k
W[:, :, 3:8] = np.moveaxis(Y, 0, -1)      # C^S = sum_q s_q Y_q


def couplet_from(L, s):
    """Couplet C (3x3) from torque L (3,) and stresslet coordinates s (5,)."""
    return np.einsum('mnq,q->mn', W, np.concatenate([L, s]))


def omega_e_from(D):
    """(Omega (3,), e (5,)) from a velocity gradient D_ij = du_i/dx_j.

    Omega_k = -1/2 eps_kij D_ij and e_q = Y_q : D, i.e. the transpose of the
    map used by couplet_from, which is what makes the grand mobility
    symmetric in the stored coordinates."""
    v = np.einsum('ijq,ij->q', W, D)
    return v[0:3], v[3:8]


def cartesian_to_11(UF, UC, DF, DC):
    """Assemble 11x11 blocks from Cartesian pair tensors.

    UF[..., i, m], UC[..., i, m, n], DF[..., i, j, m], DC[..., i, j, m, n]
    (leading batch axes allowed) with U_i = UF_im F_m + UC_imn C_mn and
    D_ij = DF_ijm F_m + DC_ijmn C_mn (Sec. II.A)."""
    batch = UF.shape[:-2]
    out = np.zeros(batch + (NCOMP, NCOMP))
    out[..., 0:3, 0:3] = UF
    out[..., 0:3, 3:11] = np.einsum('...imn,mnq->...iq', UC, W)
    out[..., 3:11, 0:3] = np.einsum('...ijm,ijq->...qm', DF, W)
    out[..., 3:11, 3:11] = np.einsum('...ijmn,ijp,mnq->...pq', DC, W, W)
    return out


# Index sets of the stored 11-vector.
IDX_U = slice(0, 3)
IDX_OMEGA = slice(3, 6)
IDX_E = slice(6, 11)
IDX_UFRAK = slice(0, 6)     # generalized velocity (U, Omega) / force (F, L)


def block_indices(N, comps):
    """Flat indices into an 11N vector for the given per-particle components."""
    comps = np.arange(NCOMP)[comps]
    return (np.arange(N)[:, None] * NCOMP + comps[None, :]).ravel()
