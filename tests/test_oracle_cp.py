"""Pins for the oracle's CP machinery (Sec. 2.1 model, Sec. 3.1 Decompose)."""

import itertools

import numpy as np
import pytest

from oracle import cp


def rand_tensor(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_unfoldings_brute_force():
    X = rand_tensor((4, 3, 5), 0)
    I, J, K = X.shape
    X1, X2, X3 = cp.unfold(X, 0), cp.unfold(X, 1), cp.unfold(X, 2)
    for i, j, k in itertools.product(range(I), range(J), range(K)):
        assert X1[i, j + J * k] == X[i, j, k]
        assert X2[j, i + I * k] == X[i, j, k]
        assert X3[k, i + I * j] == X[i, j, k]


def test_khatri_rao_columns_are_kronecker():
    g = np.random.default_rng(1)
    U, V = g.standard_normal((4, 3)), g.standard_normal((5, 3))
    KR = cp.khatri_rao(U, V)
    for r in range(3):
        np.testing.assert_array_equal(KR[:, r], np.kron(U[:, r], V[:, r]))


def test_khatri_rao_gram_identity():
    g = np.random.default_rng(2)
    A, B = g.standard_normal((7, 4)), g.standard_normal((6, 4))
    KR = cp.khatri_rao(B, A)
    np.testing.assert_allclose(KR.T @ KR, (B.T @ B) * (A.T @ A), rtol=1e-13, atol=1e-13)


def test_unfolding_of_cp_model():
    g = np.random.default_rng(3)
    A, B, C = g.standard_normal((4, 2)), g.standard_normal((3, 2)), g.standard_normal((5, 2))
    X = cp.reconstruct(A, B, C)
    np.testing.assert_allclose(cp.unfold(X, 0), A @ cp.khatri_rao(C, B).T, atol=1e-13)
    np.testing.assert_allclose(cp.unfold(X, 1), B @ cp.khatri_rao(C, A).T, atol=1e-13)
    np.testing.assert_allclose(cp.unfold(X, 2), C @ cp.khatri_rao(B, A).T, atol=1e-13)


def mttkrp_loops(X, F, mode):
    I, J, K = X.shape
    R = F[(mode + 1) % 3].shape[1]
    out = np.zeros((X.shape[mode], R))
    for i in range(I):
        for j in range(J):
            for k in range(K):
                idx = (i, j, k)
                for r in range(R):
                    p = X[i, j, k]
                    for m in range(3):
                        if m != mode:
                            p *= F[m][idx[m], r]
                    out[idx[mode], r] += p
    return out


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_mttkrp_dense_triple_loop(mode):
    X = rand_tensor((6, 5, 4), 4)
    g = np.random.default_rng(5)
    F = [g.standard_normal((6, 3)), g.standard_normal((5, 3)), g.standard_normal((4, 3))]
    np.testing.assert_allclose(cp.mttkrp_dense(X, F, mode), mttkrp_loops(X, F, mode),
                               rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_mttkrp_coo_equals_dense(mode):
    X = rand_tensor((6, 5, 4), 6)
    X[np.abs(X) < 0.7] = 0.0
    idx = np.argwhere(X != 0)
    vals = X[X != 0]
    g = np.random.default_rng(7)
    F = [g.standard_normal((6, 3)), g.standard_normal((5, 3)), g.standard_normal((4, 3))]
    np.testing.assert_allclose(cp.mttkrp_coo(idx, vals, F, mode, X.shape),
                               cp.mttkrp_dense(X, F, mode), rtol=1e-12, atol=1e-12)
    perm = np.random.default_rng(8).permutation(len(vals))
    np.testing.assert_allclose(cp.mttkrp_coo(idx[perm], vals[perm], F, mode, X.shape),
                               cp.mttkrp_dense(X, F, mode), rtol=1e-12, atol=1e-12)


def test_mttkrp_closed_form_on_exact_model():
    g = np.random.default_rng(9)
    A, B, C = g.standard_normal((8, 3)), g.standard_normal((7, 3)), g.standard_normal((6, 3))
    X = cp.reconstruct(A, B, C)
    F = [A, B, C]
    np.testing.assert_allclose(cp.mttkrp_dense(X, F, 0), A @ ((B.T @ B) * (C.T @ C)), atol=1e-11)
    np.testing.assert_allclose(cp.mttkrp_dense(X, F, 1), B @ ((A.T @ A) * (C.T @ C)), atol=1e-11)
    np.testing.assert_allclose(cp.mttkrp_dense(X, F, 2), C @ ((A.T @ A) * (B.T @ B)), atol=1e-11)


def test_solve_normal_cholesky_and_fallback():
    g = np.random.default_rng(10)
    F = g.standard_normal((30, 4))
    V = F.T @ F
    M = g.standard_normal((9, 4))
    U, used = cp.solve_normal(M, V)
    assert not used
    assert np.linalg.norm(U @ V - M) <= 1e-12 * np.linalg.norm(M)
    np.testing.assert_allclose(U, np.linalg.solve(V, M.T).T, rtol=1e-10)
    # singular V (a repeated column): pseudo-inverse fallback
    F2 = np.concatenate([F[:, :3], F[:, :1]], axis=1)
    V2 = F2.T @ F2
    U2, used2 = cp.solve_normal(M, V2)
    assert used2
    np.testing.assert_allclose(U2, M @ np.linalg.pinv(V2, rcond=4 * np.finfo(float).eps),
                               rtol=1e-8, atol=1e-10)


def test_normalize_columns_keeps_zero_column():
    U = np.array([[3.0, 0.0], [4.0, 0.0]])
    Un, n = cp.normalize_columns(U)
    np.testing.assert_array_equal(n, [5.0, 0.0])
    np.testing.assert_array_equal(Un, [[0.6, 0.0], [0.8, 0.0]])


def exact_low_rank(I, J, K, R, seed):
    g = np.random.default_rng(seed)
    A, B, C = g.random((I, R)), g.random((J, R)), g.random((K, R))
    return A, B, C, cp.reconstruct(A, B, C)


def test_cp_als_recovers_exact_low_rank():
    A, B, C, X = exact_low_rank(20, 20, 20, 3, 11)
    B0 = cp.als_init_factor(1, 0, 2, 2, 0, 0, 20, 3)
    C0 = cp.als_init_factor(1, 0, 2, 3, 0, 0, 20, 3)
    (a, b, c), lam, npinv = cp.cp_als(lambda F, m: cp.mttkrp_dense(X, F, m), X.shape, 3, 500,
                                      B0, C0)
    assert npinv == 0
    assert 1 - cp.fit_explicit(X, a, b, c, lam) < 1e-10
    assert cp.fms(a, b, c, lam, A, B, C, np.ones(3)) > 0.9999
    for M in (a, b, c):
        np.testing.assert_allclose(np.linalg.norm(M, axis=0), 1.0, rtol=1e-13)


def test_cp_als_fit_monotone():
    g = np.random.default_rng(12)
    A, B, C, X = exact_low_rank(12, 11, 10, 3, 12)
    X = X + 0.05 * g.standard_normal(X.shape)
    B0 = cp.als_init_factor(2, 0, 2, 2, 0, 0, 11, 3)
    C0 = cp.als_init_factor(2, 0, 2, 3, 0, 0, 10, 3)
    fits = []
    for it in range(1, 25):
        (a, b, c), lam, _ = cp.cp_als(lambda F, m: cp.mttkrp_dense(X, F, m), X.shape, 3, it,
                                      B0, C0)
        fits.append(cp.fit_explicit(X, a, b, c, lam))
    assert all(f2 >= f1 - 1e-12 for f1, f2 in zip(fits, fits[1:]))


def test_fit_gram_equals_explicit_residual():
    g = np.random.default_rng(13)
    X = g.standard_normal((7, 6, 5))
    A, B, C = g.standard_normal((7, 3)), g.standard_normal((6, 3)), g.standard_normal((5, 3))
    lam = g.random(3) + 0.5
    M3 = cp.mttkrp_dense(X, [A, B, C], 2)
    assert abs(cp.fit_gram(float(np.sum(X * X)), A, B, C, lam, M3)
               - cp.fit_explicit(X, A, B, C, lam)) < 1e-12


def test_sort_by_weight_stable():
    A = np.eye(3)
    lam = np.array([1.0, 3.0, 1.0])
    a, b, c, l2 = cp.sort_by_weight(A, A, A, lam)
    np.testing.assert_array_equal(l2, [3.0, 1.0, 1.0])
    np.testing.assert_array_equal(a[:, 1], [1, 0, 0])  # tie keeps lower index first


def test_fms_identity_and_permutation():
    g = np.random.default_rng(14)
    A, B, C = g.random((9, 3)), g.random((8, 3)), g.random((7, 3))
    lam = np.ones(3)
    assert abs(cp.fms(A, B, C, lam, A, B, C, lam) - 1.0) < 1e-12
    p = [2, 0, 1]
    assert abs(cp.fms(A, B, C, lam, 2 * A[:, p], B[:, p], 0.5 * C[:, p], lam) - 1.0) < 1e-12


def test_round_bf16_nearest_even():
    # against the definition: the nearest of the representable neighbours
    # (8 significant bits), ties to the one with an even last bit
    g = np.random.default_rng(5)
    x = np.concatenate([g.standard_normal(2000).astype(np.float32),
                        np.float32([1.0, -1.0, 0.0, 3.0e38, 1e-30, 1.00390625, 1.01171875,
                                    1.0078125, -1.00390625])])
    got = cp.round_bf16(x)
    for v, r in zip(x.astype(np.float64), got):
        if v == 0.0:
            assert r == 0.0
            continue
        m, e = np.frexp(abs(v))                # |v| = m 2^e, m in [0.5, 1)
        ulp = 2.0 ** (e - 8)                   # 8 significant bits
        lo = np.floor(abs(v) / ulp) * ulp
        hi = lo + ulp
        if abs(v) - lo < hi - abs(v):
            want = lo
        elif abs(v) - lo > hi - abs(v):
            want = hi
        else:
            want = lo if int(round(lo / ulp)) % 2 == 0 else hi
        assert r == np.copysign(want, v), (v, r, want)
    # exact halves: 1 + 2^-8 goes down to 1, 1 + 3 * 2^-8 goes up to 1 + 2^-6
    assert cp.round_bf16(np.float32(1.00390625)) == 1.0
    assert cp.round_bf16(np.float32(1.01171875)) == 1.015625


def test_fms_weight_penalty():
    # same unit components, weights differing by a factor: penalty 1 - |l1 - l2| / max
    g = np.random.default_rng(15)
    A, _ = cp.normalize_columns(g.random((6, 2)))
    B, _ = cp.normalize_columns(g.random((5, 2)))
    C, _ = cp.normalize_columns(g.random((4, 2)))
    lam = np.array([2.0, 1.0])
    assert abs(cp.fms(A, B, C, lam, A, B, C, 2 * lam) - 0.5) < 1e-12
    assert abs(cp.fms(A, B, C, lam, A, B, C, lam * [1.0, 3.0]) - (1.0 + 1.0 / 3.0) / 2) < 1e-12
    # weights carried by a column norm instead of lambda count the same
    A3 = A.copy()
    A3[:, 1] *= 3.0
    assert abs(cp.fms(A, B, C, lam, A3, B, C, lam) - (1.0 + 1.0 / 3.0) / 2) < 1e-12


def test_fms_worked_cosines():
    # one component: cosines 1/2 (mode 1), -1 (mode 2, sign ignored), 1 (mode 3)
    t = np.pi / 3
    A1, A2 = np.array([[1.0], [0.0]]), np.array([[np.cos(t)], [np.sin(t)]])
    B1, B2 = np.array([[1.0], [2.0]]), np.array([[-1.0], [-2.0]])
    C1 = C2 = np.array([[3.0]])
    lam = np.array([1.0])
    assert abs(cp.fms(A1, B1, C1, lam, A2, B2, C2, lam) - 0.5) < 1e-12
    # orthogonal components score 0
    assert abs(cp.fms(A1, B1, C1, lam, np.array([[0.0], [1.0]]), B2, C2, lam)) < 1e-15


def test_fms_assignment_against_all_permutations():
    # the pairing maximises the summed similarity: brute force over R! pairings
    import itertools
    g = np.random.default_rng(16)
    R = 4
    m1 = [g.random((n, R)) for n in (7, 6, 5)]
    m2 = [g.random((n, R)) for n in (7, 6, 5)]
    l1, l2 = g.random(R) + 0.5, g.random(R) + 0.5
    unit = [[M / np.linalg.norm(M, axis=0) for M in m] for m in (m1, m2)]
    w1 = l1 * np.prod([np.linalg.norm(M, axis=0) for M in m1], axis=0)
    w2 = l2 * np.prod([np.linalg.norm(M, axis=0) for M in m2], axis=0)
    best, best_sim = None, -1.0
    for perm in itertools.permutations(range(R)):
        sims = [np.prod([abs(unit[0][n][:, f] @ unit[1][n][:, perm[f]]) for n in range(3)])
                for f in range(R)]
        if sum(sims) > best_sim:
            best_sim = sum(sims)
            best = sum(s * (1 - abs(w1[f] - w2[perm[f]]) / max(w1[f], w2[perm[f]]))
                       for f, s in enumerate(sims)) / R
    assert abs(cp.fms(*m1, l1, *m2, l2) - best) < 1e-12
