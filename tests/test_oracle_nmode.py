"""Pins of the N-mode oracle (Sec. 2: the method carries over to any number of
modes) against brute force, closed forms, the third-order oracle at N = 3 and
exact recovery of noise-free low-rank data."""

import itertools

import numpy as np
import pytest

import synth
from oracle import cp, nmode
from oracle import sambaten as osb


def test_mttkrp_brute_force_order4():
    rng = np.random.default_rng(1)
    dims = (2, 3, 2, 3)
    X = rng.standard_normal(dims)
    U = [rng.standard_normal((d, 2)) for d in dims]
    for n in range(4):
        want = np.zeros((dims[n], 2))
        for idx in itertools.product(*(range(d) for d in dims)):
            for r in range(2):
                p = X[idx]
                for m in range(4):
                    if m != n:
                        p *= U[m][idx[m], r]
                want[idx[n], r] += p
        np.testing.assert_allclose(nmode.mttkrp(X, U, n), want, rtol=1e-13, atol=1e-13)


def test_mttkrp_rank_one_closed_form_order5():
    # X = u_0 o ... o u_4: M_n(:, r) = u_n * prod_{m != n} <u_m, U_m(:, r)>
    rng = np.random.default_rng(2)
    dims = (3, 4, 2, 3, 5)
    u = [rng.standard_normal(d) for d in dims]
    X = nmode.reconstruct([v[:, None] for v in u])
    U = [rng.standard_normal((d, 3)) for d in dims]
    for n in range(5):
        scal = np.ones(3)
        for m in range(5):
            if m != n:
                scal = scal * (u[m] @ U[m])
        np.testing.assert_allclose(nmode.mttkrp(X, U, n), np.outer(u[n], scal), rtol=1e-12,
                                   atol=1e-12)


def test_mttkrp_order3_is_the_unfolding_product():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4, 5, 6))
    U = [rng.standard_normal((d, 3)) for d in X.shape]
    for n in range(3):
        np.testing.assert_allclose(nmode.mttkrp(X, U, n), cp.mttkrp_dense(X, U, n), rtol=1e-12,
                                   atol=1e-12)


def test_moi_brute_force_order4():
    rng = np.random.default_rng(4)
    q = rng.integers(0, 1 << 40, size=(3, 2, 4, 3), dtype=np.uint64)
    w = nmode.moi(q)
    for m in range(4):
        want = [0] * q.shape[m]
        for idx in itertools.product(*(range(d) for d in q.shape)):
            want[idx[m]] += int(q[idx])
        assert [int(v) for v in w[m]] == want


def test_reconstruct_and_both_fits_agree():
    g = synth.DenseCPN((6, 5, 4, 7), 2, seed=5, noise=0.1, dtype=np.float64)
    X = g.slices(0, 7)
    Us, lam = g.true_model()
    # reconstruct() of the unit factors and lambda is the clean tensor
    np.testing.assert_allclose(nmode.reconstruct(Us, lam),
                               nmode.reconstruct([U for U in g.U]), rtol=1e-12, atol=1e-12)
    cfg = nmode.Config(rank=2, reps=1, als_iters=1, sample_factor=1, seed=1, order=4)
    o = nmode.OracleTensorN(cfg, X, factors=Us, lam=lam)
    assert abs(o.fit() - o.fit_explicit()) < 1e-10
    assert 0.8 < o.fit() < 0.99


def test_cp_als_recovers_exact_low_rank_order4():
    g = synth.DenseCPN((9, 8, 7, 10), 3, seed=6, noise=0.0, dtype=np.float64)
    X = g.slices(0, 10)
    cfg = nmode.Config(rank=3, reps=1, als_iters=1, sample_factor=1, seed=2, order=4,
                       init_iters=300)
    o = nmode.OracleTensorN(cfg, X)
    assert o.fit_explicit() > 1.0 - 1e-8
    assert np.all(np.diff(o.lam) <= 0)  # sorted by weight
    # the components are the true ones up to order and sign
    Ut, lt = g.true_model()
    for U, V in zip(o.U, Ut):
        cos = np.abs(U.T @ V)
        np.testing.assert_allclose(np.sort(cos.max(axis=1)), 1.0, atol=1e-6)
    np.testing.assert_allclose(np.sort(o.lam), np.sort(lt), rtol=1e-6)


@pytest.mark.parametrize("bf16", [False, True])
def test_order3_update_is_the_third_order_update(bf16):
    # the same configuration through both oracles: identical up to rounding
    # (also with the summaries rounded to bfloat16)
    g = synth.DenseCP(30, 28, 40, 4, seed=3, noise=0.05, dtype=np.float64)
    X = g.slices(0, 40)
    c3 = osb.Config(rank=4, reps=3, als_iters=15, sample_factor=(2, 3, 2), seed=5,
                    k_capacity=40, init_iters=30, summary_bf16=bf16)
    cn = nmode.Config(rank=4, reps=3, als_iters=15, sample_factor=(2, 3, 2), seed=5, order=3,
                      k_capacity=40, init_iters=30, summary_bf16=bf16)
    o3 = osb.OracleTensor(c3, osb.DENSE, (30, 28, 30), X0=X[:, :, :30])
    on = nmode.OracleTensorN(cn, X[:, :, :30])
    for a, b in zip((o3.A, o3.B, o3.C, o3.lam), (*on.U, on.lam)):
        np.testing.assert_allclose(b, a, rtol=1e-10, atol=1e-12)
    for b in range(2):
        Y = X[:, :, 30 + 5 * b:35 + 5 * b]
        d3 = o3.update(Y, debug=True)
        dn = on.update(Y, debug=True)
        for r3, rn in zip(d3["reps"], dn["reps"]):
            for key, m in (("Is", 0), ("Js", 1), ("Ks", 2)):
                np.testing.assert_array_equal(rn["S"][m], r3[key])
            np.testing.assert_array_equal(rn["pi"], r3["pi"])
        for a, c in zip((o3.A, o3.B, o3.C), on.U):
            np.testing.assert_allclose(c, a, rtol=1e-10, atol=1e-12)
        assert abs(o3.fit() - on.fit()) < 1e-12
    if bf16:  # the rounding is applied: FP64 summaries give other new rows
        cf = nmode.Config(rank=4, reps=3, als_iters=15, sample_factor=(2, 3, 2), seed=5,
                          order=3, k_capacity=40, init_iters=30)
        of = nmode.OracleTensorN(cf, X[:, :, :30])
        for b in range(2):
            of.update(X[:, :, 30 + 5 * b:35 + 5 * b])
        assert np.max(np.abs(of.U[2][30:] - on.U[2][30:])) > 1e-6


@pytest.mark.parametrize("dims,R,flip", [((12, 10, 9, 30), 3, (1, 2)),
                                         ((8, 7, 6, 5, 20), 2, (0, 4))])
def test_exact_data_update_recovers_the_true_new_rows(dims, R, flip):
    """Noise-free rank-R data and the true model: every step of the update is
    exact up to the ALS convergence, so the new last-mode rows are the true
    ones.  Component 0 has its sign flipped in two modes of the given model
    (the tensor is unchanged); the matching must undo it in the summary
    factors, so a sign or scale slip anywhere shows in the new rows."""
    g = synth.DenseCPN(dims, R, seed=2, noise=0.0, dtype=np.float64)
    K = dims[-1]
    K0 = K - 6
    X = g.slices(0, K)
    Us, lam = g.true_model_prefix(K0)
    for m in flip:
        Us[m][:, 0] *= -1.0
    cfg = nmode.Config(rank=R, reps=4, als_iters=300, sample_factor=2, seed=9, order=len(dims),
                       k_capacity=K)
    o = nmode.OracleTensorN(cfg, X[..., :K0], factors=Us, lam=lam)
    d = o.update(X[..., K0:], debug=True)
    Ut, _ = g.true_model()
    want = Ut[-1][K0:].copy()
    if len(dims) - 1 in flip:
        want[:, 0] *= -1.0
    np.testing.assert_allclose(d["C_new"], want, atol=1e-8)
    assert d["n"] == [-(-D // 2) for D in dims[:-1]] + [-(-K0 // 2)]
    # the sample factors came out in some other column order in at least one repetition
    assert any(np.any(r["pi"] != np.arange(R)) for r in d["reps"]) or R == 2
    assert o.fit_explicit() > 1.0 - 1e-7


def test_summary_is_the_restriction_and_samples_are_sorted():
    g = synth.DenseCPN((7, 6, 5, 12), 2, seed=8, noise=0.2, dtype=np.float64)
    X = g.slices(0, 12)
    cfg = nmode.Config(rank=2, reps=2, als_iters=3, sample_factor=(2, 3, 1, 2), seed=4,
                       order=4, k_capacity=12)
    o = nmode.OracleTensorN(cfg, X[..., :9], factors=g.true_model_prefix(9)[0],
                            lam=g.true_model()[1])
    d = o.update(X[..., 9:], debug=True)
    assert d["n"] == [4, 2, 5, 5]
    for r in d["reps"]:
        S = r["S"]
        for m, s in enumerate(S):
            assert np.all(np.diff(s) > 0)
            assert len(s) == d["n"][m]
        Kp = list(S[-1]) + [9, 10, 11]
        for idx in itertools.product(*(range(len(s)) for s in S[:-1]), range(len(Kp))):
            src = tuple(S[m][idx[m]] for m in range(3)) + (Kp[idx[3]],)
            assert r["Z"][idx] == X[src]


def test_zero_entry_is_filled_from_the_repetitions():
    g = synth.DenseCPN((10, 9, 8, 16), 2, seed=12, noise=0.0, dtype=np.float64)
    X = g.slices(0, 16)
    Us, lam = g.true_model_prefix(12)
    truth = Us[1][3, 1]
    Us[1][3, 1] = 0.0
    cfg = nmode.Config(rank=2, reps=3, als_iters=200, sample_factor=(2, 1, 2, 2), seed=3,
                       order=4, k_capacity=16)
    o = nmode.OracleTensorN(cfg, X[..., :12], factors=Us, lam=lam)
    o.update(X[..., 12:])
    # every repetition samples all of mode 1 (s = 1); the filled value is the
    # true entry in units of the anchor column, which lost one entry
    scale = np.linalg.norm(Us[1][:, 1]) / np.linalg.norm(g.true_model()[0][1][:, 1])
    assert o.U[1][3, 1] == pytest.approx(truth * scale, rel=1e-6)
    # entries that were not zero are untouched
    keep = np.ones_like(Us[1], dtype=bool)
    keep[3, 1] = False
    np.testing.assert_array_equal(o.U[1][keep], Us[1][keep])


def test_non_finite_batch_is_refused_without_change():
    g = synth.DenseCPN((5, 4, 3, 8), 2, seed=1, noise=0.1, dtype=np.float64)
    X = g.slices(0, 8)
    cfg = nmode.Config(rank=2, reps=2, als_iters=3, sample_factor=2, seed=1, order=4,
                       k_capacity=8)
    o = nmode.OracleTensorN(cfg, X[..., :6], factors=g.true_model_prefix(6)[0],
                            lam=g.true_model()[1])
    Y = X[..., 6:].copy()
    Y[1, 2, 0, 1] = np.nan
    with pytest.raises(osb.NumericError):
        o.update(Y)
    assert o.dims[-1] == 6 and o.t == 0
