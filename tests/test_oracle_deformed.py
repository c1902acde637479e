"""Pins of the oracle on deformed periodic lattices (Sec. II.C.2): lattice
vectors L A e_i for a volume-preserving A (Lees-Edwards shear, planar
extension).  The exact sums are checked against what the mathematics fixes:

* M_w + M_r does not depend on the splitting parameter xi, block by block
  (a wrong reciprocal lattice -- A instead of A^-T -- or a wrong image set
  breaks this);
* a shear by gamma = 1 maps the cubic lattice onto itself (a lattice vector
  L (e_x + e_y) replaces L e_y), so both sums equal the cube's;
* M_w is symmetric positive semi-definite;
* lambda_max of Eqs. lmax1, lmax2 from the definition (Table 1 is pinned with
  the support rule in test_oracle_pins).
"""
import numpy as np
import pytest

from oracle import ewald, params

X4 = np.array([[1.0, 1.0, 1.0], [3.1, 1.2, 0.8], [1.5, 4.0, 5.5], [7.9, 8.5, 0.3]])
L = 9.0


@pytest.mark.parametrize('A', [params.shear_tensor(0.5), params.shear_tensor(-0.3),
                               params.extension_tensor(1.5)],
                         ids=['shear0.5', 'shear-0.3', 'ext1.5'])
def test_deformed_sum_independent_of_xi(A):
    M1 = ewald.grand_dense(X4, L, 0.6, A=A)
    M2 = ewald.grand_dense(X4, L, 0.9, A=A)
    scale = np.abs(M1).max()
    for b in range(4):
        for c in range(4):
            blk = (slice(11 * b, 11 * b + 11), slice(11 * c, 11 * c + 11))
            assert np.abs(M1[blk] - M2[blk]).max() < 1e-12 * scale, (b, c)


def test_unit_shear_is_the_cube():
    x = X4
    for part in (ewald.wave_dense, ewald.real_dense):
        M0 = part(x, L, 0.7)
        M1 = part(x, L, 0.7, A=params.shear_tensor(1.0))
        assert np.abs(M0 - M1).max() < 1e-12 * np.abs(M0).max(), part.__name__


def test_deformation_changes_the_sum():
    """The check above is not vacuous: gamma = 0.5 differs from the cube."""
    M0 = ewald.grand_dense(X4, L, 0.7)
    M1 = ewald.grand_dense(X4, L, 0.7, A=params.shear_tensor(0.5))
    assert np.abs(M0 - M1).max() > 1e-4 * np.abs(M0).max()


def test_deformed_wave_part_spsd():
    M = ewald.wave_dense(X4, L, 0.7, A=params.shear_tensor(0.5))
    assert np.abs(M - M.T).max() < 1e-14 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > -1e-12 * np.abs(M).max()


def test_matrix_free_equals_dense_on_deformed_lattice():
    A = params.extension_tensor(1.5)
    q = np.random.default_rng(2).normal(size=(4, 11))
    for dense, apply in ((ewald.wave_dense, ewald.wave_apply),
                         (ewald.real_dense, ewald.real_apply)):
        y1 = dense(X4, L, 0.7, A=A) @ q.reshape(-1)
        y2 = apply(X4, q, L, 0.7, A=A).reshape(-1)
        assert np.abs(y1 - y2).max() < 1e-12 * np.abs(y1).max()


def test_non_volume_preserving_deformation_refused():
    with pytest.raises(ValueError):
        ewald.wave_dense(X4, L, 0.7, A=np.diag([1.1, 1.0, 1.0]))


@pytest.mark.parametrize('g', [0.1, 0.5, 1.0, 2.0])
def test_lambda_max_closed_forms(g):
    assert params.lambda_max(params.shear_tensor(g)) == pytest.approx(
        1 + g * g / 2 + g * np.sqrt(1 + g * g / 4), rel=1e-13)
    e = 1.0 + g
    assert params.lambda_max(params.extension_tensor(e)) == pytest.approx(e * e, rel=1e-13)
    assert params.lambda_max(params.extension_tensor(1 / e)) == pytest.approx(e * e, rel=1e-13)
