"""Pins of the oracle's core consistency diagnostic and GetRank (Sec. 3.2)."""

import numpy as np

from oracle import cp
from oracle import sambaten as osb


def _model(dims, R, seed):
    g = np.random.default_rng(seed)
    F = [cp.normalize_columns(g.random((n, R)))[0] for n in dims]
    lam = g.random(R) + 1.0
    return F, lam


def test_corcondia_worked_examples():
    # superdiagonal 2x2x2 tensor with identity factors: the core is the tensor itself
    Z = np.zeros((2, 2, 2))
    Z[0, 0, 0] = Z[1, 1, 1] = 1.0
    I2 = np.eye(2)
    assert abs(cp.corcondia(Z, I2, I2, I2, np.ones(2)) - 100.0) < 1e-12
    # all-ones 2x2x2 (rank one) with the same two-component model: G = Z, the six
    # off-superdiagonal ones and the two matched ones give 100 (1 - 6 / 2) = -200
    assert abs(cp.corcondia(np.ones((2, 2, 2)), I2, I2, I2, np.ones(2)) + 200.0) < 1e-12
    # weights scale the core: lambda = 2 on an exact rank-one tensor still gives 100
    a = np.array([[0.6], [0.8]])
    Z1 = 2.0 * np.einsum("i,j,k->ijk", a[:, 0], a[:, 0], a[:, 0])
    assert abs(cp.corcondia(Z1, a, a, a, np.array([2.0])) - 100.0) < 1e-12


def test_corcondia_exact_low_rank_is_100():
    (A, B, C), lam = _model((9, 8, 7), 3, 1)
    Z = cp.reconstruct(A, B, C, lam)
    assert abs(cp.corcondia(Z, A, B, C, lam) - 100.0) < 1e-9


def test_corcondia_core_against_kronecker_form():
    # vec(G) = (pinv(C') kron pinv(B) kron pinv(A)) vec(Z) in column-major order
    g = np.random.default_rng(2)
    Z = g.standard_normal((5, 4, 3))
    A, B, C = g.random((5, 2)), g.random((4, 2)), g.random((3, 2))
    lam = np.array([1.5, 0.5])
    Kr = np.kron(np.linalg.pinv(C * lam), np.kron(np.linalg.pinv(B), np.linalg.pinv(A)))
    G = (Kr @ Z.reshape(-1, order="F")).reshape((2, 2, 2), order="F")
    T = np.zeros((2, 2, 2))
    T[0, 0, 0] = T[1, 1, 1] = 1.0
    want = 100.0 * (1.0 - np.sum((G - T) ** 2) / 2)
    assert abs(cp.corcondia(Z, A, B, C, lam) - want) < 1e-9


def _init(dims, seed):
    g = np.random.default_rng(seed)

    def init(i, q):
        return g.random((dims[1], i)), g.random((dims[2], i))
    return init


def test_get_rank_finds_the_rank_of_noiseless_data():
    (A, B, C), lam = _model((12, 11, 10), 2, 3)
    Z = cp.reconstruct(A, B, C, lam)
    Rn, F, l, cc = cp.get_rank(Z, 4, 2, 90.0, 60, _init(Z.shape, 4))
    assert Rn == 2
    assert max(cc[0]) > 99.999 and max(cc[1]) > 99.9
    assert max(cc[2]) < 90.0 and max(cc[3]) < 90.0
    # the kept run is the best one at rank 2 and fits the data
    assert F[0].shape == (12, 2)
    assert np.linalg.norm(cp.reconstruct(*F, l) - Z) < 1e-2 * np.linalg.norm(Z)


def test_get_rank_threshold_edges():
    (A, B, C), lam = _model((8, 7, 6), 3, 5)
    Z = cp.reconstruct(A, B, C, lam) + 0.01 * np.random.default_rng(6).standard_normal((8, 7, 6))
    # nothing reaches the threshold: rank one is still returned
    assert cp.get_rank(Z, 3, 1, 1e9, 20, _init(Z.shape, 7))[0] == 1
    # every rank qualifies: the largest candidate
    assert cp.get_rank(Z, 3, 1, -1e9, 20, _init(Z.shape, 7))[0] == 3


def test_match_leaves_components_without_partner():
    # two sample columns for three current components: the best two pairs
    g = np.random.default_rng(8)
    A, B, C = g.random((6, 3)), g.random((5, 3)), g.random((4, 3))
    Ap, Bp, Cp = A[:, [2, 0]], B[:, [2, 0]], C[:, [2, 0]]
    pi = osb.match(A, B, C, Ap, Bp, Cp)[0]
    np.testing.assert_array_equal(pi, [1, -1, 0])
