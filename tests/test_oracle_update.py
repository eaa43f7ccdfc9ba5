"""Pins for the oracle's batch update (Algorithm 1, Sec. 3.1)."""

import itertools

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import cp, rng
from oracle import sambaten as sb


def exact_model(I, J, K, R, seed):
    g = np.random.default_rng(seed)
    A, B, C = g.random((I, R)), g.random((J, R)), g.random((K, R))
    X = cp.reconstruct(A, B, C)
    return A, B, C, X


def unit_model(A, B, C, K0):
    nA, nB, nC = (np.linalg.norm(M, axis=0) for M in (A, B, C[:K0]))
    return A / nA, B / nB, C[:K0] / nC, nA * nB * nC, nC


@pytest.mark.parametrize("R", [2, 3, 4, 5, 6])
def test_assignment_equals_brute_force(R):
    g = np.random.default_rng(R)
    for _ in range(5):
        S = g.random((R, R))
        rows, cols = linear_sum_assignment(S, maximize=True)
        best = max(sum(S[f, p[f]] for f in range(R)) for p in itertools.permutations(range(R)))
        assert abs(S[rows, cols].sum() - best) < 1e-12


def test_lemma1_matched_cosines_are_one():
    # Lemma 1: unit columns of the same latent factor have inner product 1,
    # different ones have inner product < 1.
    g = np.random.default_rng(1)
    R = 4
    A, B, C = g.random((12, R)), g.random((11, R)), g.random((10, R))
    perm = np.array([2, 0, 3, 1])
    scale = np.array([3.0, 0.5, 2.0, 7.0])
    pi, sigA, sigB, nA, nB, S, cosA, cosB = sb.match(
        A, B, C, A[:, perm] * scale, B[:, perm] / scale, C[:, perm])
    inv = np.argsort(perm)
    np.testing.assert_array_equal(pi, inv)
    for f in range(R):
        assert abs(cosA[f, pi[f]] - 1) < 1e-12 and abs(cosB[f, pi[f]] - 1) < 1e-12
        for g2 in range(R):
            if g2 != pi[f]:
                assert cosA[f, g2] < 1 - 1e-6
    np.testing.assert_array_equal(sigA, 1.0)


def test_match_recovers_signs():
    g = np.random.default_rng(2)
    R = 3
    A, B, C = g.standard_normal((9, R)), g.standard_normal((8, R)), g.standard_normal((7, R))
    flip = np.array([-1.0, 1.0, -1.0])
    pi, sigA, sigB, *_ = sb.match(A, B, C, A * flip, B * flip, C)
    np.testing.assert_array_equal(pi, np.arange(R))
    np.testing.assert_array_equal(sigA, flip)
    np.testing.assert_array_equal(sigB, flip)


def make_dense(I, J, K0, Kn, R, seed, noise, reps, iters, s=2, batches=1):
    A, B, C, X = exact_model(I, J, K0 + batches * Kn, R, seed)
    if noise:
        X = X + noise * np.random.default_rng(seed + 100).standard_normal(X.shape)
    a, b, c, lam, nC = unit_model(A, B, C, K0)
    cfg = sb.Config(rank=R, reps=reps, als_iters=iters, sample_factor=s, seed=seed,
                    k_capacity=K0 + batches * Kn)
    T = sb.OracleTensor(cfg, sb.DENSE, (I, J, K0), X0=X[:, :, :K0], factors=(a, b, c, lam))
    return T, X, C / nC


def test_row_solve_is_rescaled_last_als_mode():
    # The new rows of C are the least-squares rows against the matched sample
    # factors; because C' comes from the last ALS mode update, they equal
    # lambda'_pi(f) C'(:, pi(f)) / (sigA sigB ||A(I_s,f)|| ||B(J_s,f)||) / lambda_f.
    T, X, _ = make_dense(20, 18, 16, 6, 3, 3, 0.02, 2, 15)
    d = T.update(X[:, :, 16:22], debug=True)
    lam = T.lam
    for r in d["reps"]:
        pi = r["pi"]
        scale = r["sigA"] * r["sigB"] * r["nA"] * r["nB"] * lam
        expected = r["Cp"][:, pi] * r["lamp"][pi] / scale
        np.testing.assert_allclose(r["Ct"], expected, rtol=1e-8, atol=1e-10)


def test_noise_free_update_recovers_new_rows():
    # Exact rank-3 data, the current model equal to the truth: every summary is
    # exactly rank 3, so after converged ALS the appended rows are the true ones.
    T, X, Ctrue = make_dense(30, 30, 30, 10, 3, 1, 0.0, 3, 1000, batches=2)
    T.update(X[:, :, 30:40])
    T.update(X[:, :, 40:50])
    assert T.K == 50 and T.t == 2
    np.testing.assert_allclose(T.C[30:], Ctrue[30:], atol=1e-9)
    assert 1 - T.fit_explicit() < 1e-9


def test_single_full_sample_reduces_to_full_cp_als():
    # s = 1, r = 1: the summary is the whole tensor, so the update is CP-ALS on
    # X u Y from the same initial factors, then match and row least squares.
    I, J, K0, Kn, R = 10, 9, 8, 4, 2
    T, X, _ = make_dense(I, J, K0, Kn, R, 4, 0.01, 1, 40, s=1)
    d = T.update(X[:, :, K0:K0 + Kn], debug=True)
    r = d["reps"][0]
    np.testing.assert_array_equal(r["Is"], np.arange(I))
    np.testing.assert_array_equal(r["Js"], np.arange(J))
    np.testing.assert_array_equal(r["Ks"], np.arange(K0))
    XY = X[:, :, :K0 + Kn]
    B0 = cp.als_init_factor(4, 0, rng.TAG_ALSINIT, 2, 0, 0, J, R)
    C0 = cp.als_init_factor(4, 0, rng.TAG_ALSINIT, 3, 0, 0, K0 + Kn, R)
    (a, b, c), lam, _ = cp.cp_als(lambda F, m: cp.mttkrp_dense(XY, F, m), XY.shape, R, 40, B0, C0)
    np.testing.assert_allclose(r["Ap"], a, atol=1e-12)
    np.testing.assert_allclose(r["Cp"], c, atol=1e-12)
    np.testing.assert_allclose(r["lamp"], lam, rtol=1e-12)


def test_zero_entries_filled_from_sampled_rows_only():
    T, X, _ = make_dense(16, 14, 12, 4, 2, 5, 0.01, 3, 20)
    zero_rows = [1, 5, 9, 13]
    A_before = T.A.copy()
    T.A[zero_rows, 1] = 0.0
    d = T.update(X[:, :, 12:16], debug=True)
    covered = set()
    for r in d["reps"]:
        covered |= set(int(i) for i in r["Is"])
    assert any(i in covered for i in zero_rows)
    for i in zero_rows:
        vals = [r["At"][np.searchsorted(r["Is"], i), 1] for r in d["reps"]
                if i in set(int(v) for v in r["Is"]) and r["valid"][1]]
        if i in covered:
            assert T.A[i, 1] == pytest.approx(np.mean(vals), rel=1e-12)
            assert T.A[i, 1] != 0.0
        else:
            assert T.A[i, 1] == 0.0
    # non-zero entries are untouched
    mask = np.ones_like(A_before, dtype=bool)
    mask[zero_rows, 1] = False
    np.testing.assert_array_equal(T.A[mask], A_before[mask])


def test_new_rows_are_mean_over_repetitions():
    T, X, _ = make_dense(16, 14, 12, 4, 3, 6, 0.01, 4, 10)
    d = T.update(X[:, :, 12:16], debug=True)
    acc = sum(r["Ct"][len(r["Ks"]):] for r in d["reps"])
    np.testing.assert_allclose(T.C[12:], acc / 4, rtol=1e-13)


def test_numeric_error_leaves_state_unchanged():
    T, X, _ = make_dense(10, 9, 8, 3, 2, 7, 0.01, 2, 5)
    Y = X[:, :, 8:11].copy()
    Y[3, 4, 1] = np.nan
    A, C, w = T.A.copy(), T.C.copy(), [v.copy() for v in T.w]
    with pytest.raises(sb.NumericError):
        T.update(Y)
    assert T.K == 8 and T.t == 0
    np.testing.assert_array_equal(T.A, A)
    np.testing.assert_array_equal(T.C, C)
    for a, b in zip(T.w, w):
        np.testing.assert_array_equal(a, b)
    T.update(X[:, :, 8:11])
    assert T.K == 11 and T.t == 1


def test_incremental_moi_equals_from_scratch():
    T, X, _ = make_dense(10, 9, 8, 3, 2, 8, 0.01, 2, 5, batches=2)
    T.update(X[:, :, 8:11])
    T.update(X[:, :, 11:14])
    q, ok = sb.quantize_sq(X[:, :, :14], T.S, T.n_max)
    assert ok
    for a, b in zip(T.w, sb.moi_dense(q)):
        np.testing.assert_array_equal(a, b)


def test_coo_update_equals_dense_update():
    # The same tensor held densely and as COO (its nonzeros): identical samples,
    # identical summaries, hence the same update up to summation order.
    I, J, K0, Kn, R = 12, 11, 10, 4, 2
    A, B, C, X = exact_model(I, J, K0 + Kn, R, 9)
    X = X + 0.01 * np.random.default_rng(9).standard_normal(X.shape)
    X[np.random.default_rng(10).random(X.shape) < 0.3] = 0.0
    a, b, c, lam, _ = unit_model(A, B, C, K0)
    cfg = sb.Config(rank=R, reps=2, als_iters=15, sample_factor=2, seed=9, k_capacity=K0 + Kn)
    Td = sb.OracleTensor(cfg, sb.DENSE, (I, J, K0), X0=X[:, :, :K0], factors=(a, b, c, lam))
    X0 = X[:, :, :K0]
    idx0 = np.argwhere(X0 != 0)
    Tc = sb.OracleTensor(cfg, sb.COO, (I, J, K0), coo0=(idx0, X0[X0 != 0]),
                         factors=(a, b, c, lam))
    assert Td.S == Tc.S
    Y = X[:, :, K0:]
    yidx = np.argwhere(Y != 0)
    dd = Td.update(Y, debug=True)
    dc = Tc.update(coo=(yidx, Y[Y != 0], Kn), debug=True)
    for rd, rc in zip(dd["reps"], dc["reps"]):
        for key in ("Is", "Js", "Ks", "pi"):
            np.testing.assert_array_equal(rd[key], rc[key])
    np.testing.assert_allclose(Tc.C, Td.C, rtol=1e-9, atol=1e-11)
    assert abs(Tc.fit() - Td.fit()) < 1e-10


def test_fit_after_update_matches_explicit():
    T, X, _ = make_dense(14, 13, 12, 4, 3, 11, 0.02, 3, 10)
    T.update(X[:, :, 12:16])
    assert abs(T.fit() - T.fit_explicit()) < 1e-7


def _persist_run(persist, refresh, batches=3, noise=0.0, iters=25):
    I, J, K0, Kn, R = 20, 18, 16, 4, 3
    A, B, C, X = exact_model(I, J, K0 + batches * Kn, R, 31)
    if noise:
        X = X + noise * np.random.default_rng(32).standard_normal(X.shape)
    An, Bn, Cn, lam, nC = unit_model(A, B, C, K0)
    cfg = sb.Config(rank=R, reps=3, als_iters=iters, sample_factor=2, seed=33,
                    k_capacity=K0 + batches * Kn, persist_summaries=persist,
                    summary_refresh=refresh)
    t = sb.OracleTensor(cfg, sb.DENSE, (I, J, K0), X0=X[:, :, :K0], factors=(An, Bn, Cn, lam))
    out = [t.update(X[:, :, K0 + b * Kn:K0 + (b + 1) * Kn], debug=True) for b in range(batches)]
    return t, out, (A, B, C, nC, K0)


def test_persistent_summaries_keep_the_sample():
    t, out, _ = _persist_run(True, 0)
    for d in out[1:]:
        for rho in range(3):
            for key in ("Is", "Js", "Ks"):
                np.testing.assert_array_equal(d["reps"][rho][key], out[0]["reps"][rho][key])
    # refresh every update: each update samples afresh and starts cold, which
    # is the plain update
    t1, out1, _ = _persist_run(True, 1, noise=0.01)
    t0, out0, _ = _persist_run(False, 0, noise=0.01)
    for d1, d0 in zip(out1, out0):
        for rho in range(3):
            for key in ("Is", "Js", "Ks"):
                np.testing.assert_array_equal(d1["reps"][rho][key], d0["reps"][rho][key])
    np.testing.assert_array_equal(t1.C, t0.C)


def test_persistent_warm_start_on_exact_data():
    # noise-free data and the true model: the kept summary factors are exact,
    # the warm-started ALS stays there and every batch's new rows come out exact
    t, out, (A, B, C, nC, K0) = _persist_run(True, 0, iters=2000)
    want = C[K0:] / nC[None, :]
    assert np.abs(t.C[K0:] - want).max() < 1e-10 * np.abs(want).max()
    # at a fixed number of sweeps the warm-started updates end closer to the truth
    tw, _, _ = _persist_run(True, 0, iters=600)
    tc, _, _ = _persist_run(False, 0, iters=600)
    assert np.abs(tw.C[K0:] - want).max() < 0.1 * np.abs(tc.C[K0:] - want).max()
    # the second update starts from the first update's summary factors
    r0, r1 = out[0]["reps"][0], out[1]["reps"][0]
    Bp0 = r0["Bp"]
    cos = np.abs(np.sum(cp.normalize_columns(r1["Bp"])[0] * Bp0, axis=0))
    assert np.all(cos > 1 - 1e-9)


def test_worker_threads_change_nothing():
    # repetitions on a thread pool and importance / fit over blocks of slices on
    # it: the same samples, matchings and importance, factors and fit to rounding
    g = np.random.default_rng(12)
    I, J, K0, Kn, R = 30, 26, 70, 6, 3
    X = g.random((I, J, K0 + 2 * Kn))
    X[3, 4, 5] = 0.0
    out = []
    for workers in (1, 4):
        cfg = sb.Config(rank=R, reps=5, als_iters=8, sample_factor=2, seed=9,
                        k_capacity=K0 + 2 * Kn, workers=workers)
        o = sb.OracleTensor(cfg, sb.DENSE, (I, J, K0), X0=X[:, :, :K0])
        ds = [o.update(X[:, :, K0 + b * Kn:K0 + (b + 1) * Kn], debug=True) for b in range(2)]
        out.append((o, ds))
    (o1, d1), (o4, d4) = out
    for w1, w4 in zip(o1.w, o4.w):
        assert np.array_equal(w1, w4)
    for a, b in zip(d1, d4):
        for r1, r4 in zip(a["reps"], b["reps"]):
            for key in ("Is", "Js", "Ks", "pi", "valid"):
                assert np.array_equal(r1[key], r4[key]), key
    for M1, M4 in ((o1.A, o4.A), (o1.B, o4.B), (o1.C, o4.C)):
        np.testing.assert_allclose(M1, M4, rtol=1e-10, atol=1e-12)
    assert abs(o1.fit() - o4.fit()) < 1e-12


def test_lambda_average_is_invariant_on_exact_data():
    # noise-free rank-R data: every summary recovers the restriction of the model,
    # so the new weight equals lambda whatever scale the given model splits between
    # lambda and C, and the paper's average leaves lambda as it was
    I, J, K0, Kn, R = 24, 22, 20, 4, 3
    A, B, C, X = exact_model(I, J, K0 + Kn, R, 14)
    An, Bn, Cn, lam, _ = unit_model(A, B, C, K0)
    for scale in (1.0, 2.0, 0.25):
        cfg = sb.Config(rank=R, reps=3, als_iters=1000, sample_factor=2, seed=14,
                        k_capacity=K0 + Kn, lambda_avg=True)
        o = sb.OracleTensor(cfg, sb.DENSE, (I, J, K0), X0=X[:, :, :K0],
                            factors=(An, Bn, Cn / scale, lam * scale))
        d = o.update(X[:, :, K0:], debug=True)
        for r in d["reps"]:
            np.testing.assert_allclose(r["lhat"], lam * scale, rtol=1e-6)
        np.testing.assert_allclose(o.lam, lam * scale, rtol=1e-6)
        assert o.fit() > 1 - 1e-6


def test_lambda_average_moves_halfway():
    # a model whose weights are wrong by a factor (A, B, C right): the summaries see
    # the true weights, so lambda moves half way towards them
    I, J, K0, Kn, R = 24, 22, 20, 4, 3
    A, B, C, X = exact_model(I, J, K0 + Kn, R, 15)
    An, Bn, Cn, lam, _ = unit_model(A, B, C, K0)
    off = np.array([2.0, 0.5, 1.0])
    cfg = sb.Config(rank=R, reps=3, als_iters=1000, sample_factor=2, seed=15,
                    k_capacity=K0 + Kn, lambda_avg=True)
    o = sb.OracleTensor(cfg, sb.DENSE, (I, J, K0), X0=X[:, :, :K0],
                        factors=(An, Bn, Cn, lam * off))
    o.update(X[:, :, K0:])
    np.testing.assert_allclose(o.lam, 0.5 * (lam * off + lam), rtol=1e-6)
    cfg0 = sb.Config(rank=R, reps=3, als_iters=1000, sample_factor=2, seed=15,
                     k_capacity=K0 + Kn)
    o0 = sb.OracleTensor(cfg0, sb.DENSE, (I, J, K0), X0=X[:, :, :K0],
                         factors=(An, Bn, Cn, lam * off))
    o0.update(X[:, :, K0:])
    np.testing.assert_array_equal(o0.lam, lam * off)
