"""Pins of the oracle's core consistency diagnostic and GetRank (Sec. 3.2)."""

import numpy as np

import synth
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


def test_corcondia_over_entries_equals_the_dense_form():
    # the core summed nonzero by nonzero is the dense core of the same tensor;
    # duplicate coordinates add up as the tensor's entry
    g = np.random.default_rng(9)
    dims = (7, 6, 5)
    X = np.where(g.random(dims) < 0.3, g.standard_normal(dims), 0.0)
    idx = np.argwhere(X != 0.0)
    vals = X[tuple(idx.T)]
    for R in (1, 2, 3):
        F = [g.random((n, R)) for n in dims]
        lam = g.random(R) + 0.5
        want = cp.corcondia(X, *F, lam)
        assert abs(cp.corcondia_coo(idx, vals, dims, *F, lam) - want) < 1e-9 * max(1, abs(want))
        half = np.concatenate([vals[:1] / 2, vals])
        idx2 = np.concatenate([idx[:1], idx])
        half[1] = vals[0] / 2
        assert abs(cp.corcondia_coo(idx2, half, dims, *F, lam) - want) < 1e-9 * max(1, abs(want))


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


def test_get_rank_on_coo_summaries_equals_dense():
    # the same sparse tensor stored both ways: GetRank on the COO summaries
    # (CP-ALS over the entries, the core consistency of the tensor they hold)
    # decides and computes what it does on the dense summaries
    I, J, K0, Kn, R, reps = 30, 26, 24, 6, 4, 3
    gen = synth.SparseSupportCP(I, J, K0 + Kn, 2, 61)
    X = gen.dense(0, K0 + Kn)
    assert 0.05 < np.count_nonzero(X) / X.size < 0.6
    g = np.random.default_rng(62)
    F = [cp.normalize_columns(g.random((n, R)))[0] for n in (I, J, K0)]
    model = (F[0], F[1], F[2], np.ones(R))
    out = []
    for fmt in (osb.DENSE, osb.COO):
        cfg = osb.Config(rank=R, reps=reps, als_iters=25, sample_factor=2, seed=63,
                         k_capacity=K0 + Kn, getrank_runs=2, getrank_threshold=90.0)
        if fmt == osb.DENSE:
            ora = osb.OracleTensor(cfg, fmt, (I, J, K0), X0=X[:, :, :K0], factors=model)
            d = ora.update(X[:, :, K0:], debug=True)
        else:
            ora = osb.OracleTensor(cfg, fmt, (I, J, K0), coo0=gen.entries(0, K0),
                                   factors=model)
            yi, yv = gen.entries(K0, K0 + Kn)
            d = ora.update(coo=(yi, yv, Kn), debug=True)
        out.append((ora, d))
    (od, dd), (oc, dc) = out
    for rd, rc in zip(dd["reps"], dc["reps"]):
        for key in ("Is", "Js", "Ks", "pi", "valid"):
            np.testing.assert_array_equal(rd[key], rc[key])
        assert rd["Rnew"] == rc["Rnew"]
        np.testing.assert_allclose(np.array(rc["cc"]), np.array(rd["cc"]), rtol=1e-7, atol=1e-7)
    # rank-2 data: GetRank keeps fewer than R components
    assert all(r["Rnew"] < R for r in dd["reps"])
    for Ud, Uc in zip((od.A, od.B, od.C, od.lam), (oc.A, oc.B, oc.C, oc.lam)):
        np.testing.assert_allclose(Uc, Ud, rtol=1e-8, atol=1e-10)
