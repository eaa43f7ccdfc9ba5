"""CP model, MTTKRP and CP-ALS in plain FP64 (oracle; test infrastructure).

Conventions (the paper's unfolding label in Sec. 2.2 is garbled; the reading
used is the Kolda-Bader one, with i fastest):

* A dense tensor is a NumPy array of shape (I, J, K); element (i, j, k).
* X_(1) = A (C kr B)^T   is I x JK,  column j + J*k
* X_(2) = B (C kr A)^T   is J x IK,  column i + I*k
* X_(3) = C (B kr A)^T   is K x IJ,  column i + I*j
* khatri_rao(U, V)[:, r] = kron(U[:, r], V[:, r])  (column-wise Kronecker,
  symbol table of Sec. 2.1), so (C kr B) row k*J + j holds C[k]*B[j].
* Factor matrices are row-major (rows x R) arrays.
"""

import numpy as np
import scipy.linalg

from . import rng


def unfold(X, mode):
    """Mode-n unfolding (mode in 0, 1, 2) with the column order above."""
    I, J, K = X.shape
    if mode == 0:
        return np.asarray(X).reshape(I, J * K, order="F")
    if mode == 1:
        return np.moveaxis(np.asarray(X), 1, 0).reshape(J, I * K, order="F")
    return np.moveaxis(np.asarray(X), 2, 0).reshape(K, I * J, order="F")


def khatri_rao(U, V):
    """Column-wise Kronecker product (Sec. 2.1 symbol table)."""
    R = U.shape[1]
    assert V.shape[1] == R
    return (U[:, None, :] * V[None, :, :]).reshape(U.shape[0] * V.shape[0], R)


def reconstruct(A, B, C, lam=None):
    """Full tensor of the CP model sum_r lam_r A(:,r) o B(:,r) o C(:,r) (Sec. 2.1)."""
    if lam is None:
        lam = np.ones(A.shape[1])
    return np.einsum("ir,jr,kr,r->ijk", A, B, C, lam)


def round_bf16(x):
    """Round to the nearest bfloat16 (8-bit significand, ties to even), via
    the nearest float32 first; returned as float64.

    bfloat16 is the upper half of an IEEE binary32: rounding keeps the top 16
    bits of the float32 pattern, adding half of the dropped unit (0x8000)
    minus one, plus the kept last bit, so that exact halves go to the even
    neighbour.  Finite inputs only."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    kept = (b + np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)
    return (kept.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def mttkrp_dense(X, factors, mode):
    """Matricised tensor times Khatri-Rao product for a dense tensor.

    mode 0: X_(1) (C kr B);  mode 1: X_(2) (C kr A);  mode 2: X_(3) (B kr A).
    `factors` is [A, B, C]; the entry for `mode` itself is not read.
    """
    A, B, C = factors
    X = np.asarray(X, dtype=np.float64)
    if mode == 0:
        return unfold(X, 0) @ khatri_rao(C, B)
    if mode == 1:
        return unfold(X, 1) @ khatri_rao(C, A)
    return unfold(X, 2) @ khatri_rao(B, A)


def mttkrp_coo(idx, vals, factors, mode, dims):
    """MTTKRP for a COO tensor: the same sum, written nonzero by nonzero.

    M(i_n, r) = sum over nonzeros of v * prod_{m != n} U_m(i_m, r).
    idx is (nnz, 3) int, vals (nnz,) float.
    """
    R = factors[(mode + 1) % 3].shape[1]
    v = np.asarray(vals, dtype=np.float64)
    prod = np.ones((v.shape[0], R))
    for m in range(3):
        if m != mode:
            prod = prod * factors[m][idx[:, m]]
    contrib = prod * v[:, None]
    out = np.zeros((dims[mode], R))
    np.add.at(out, idx[:, mode], contrib)
    return out


def solve_normal(M, V):
    """U = M V^{-1} for symmetric positive (semi)definite V.

    Cholesky (LAPACK potrf/potrs through SciPy).  If a pivot is not positive,
    fall back to the pseudo-inverse with cut-off R * eps * sigma_max.
    Returns (U, used_pinv).
    """
    R = V.shape[0]
    try:
        c = scipy.linalg.cho_factor(V, lower=True, check_finite=True)
        return scipy.linalg.cho_solve(c, M.T, check_finite=False).T, False
    except (np.linalg.LinAlgError, scipy.linalg.LinAlgError):
        P = np.linalg.pinv(V, rcond=R * np.finfo(np.float64).eps)
        return M @ P, True


def normalize_columns(U):
    """Unit 2-norm columns; a zero column stays zero.  Returns (U_n, norms)."""
    n = np.sqrt(np.sum(U * U, axis=0))
    out = U.copy()
    nz = n > 0
    out[:, nz] = out[:, nz] / n[nz]
    return out, n


def als_init_factor(seed, tensor_id, stream, mode, rep, t, rows, R, col0=0):
    """U[0,1) initial factor: entry (row, col) from Philox counter
    (row, col0 + col, tag(stream, mode, rep), t)."""
    rr, cc = np.meshgrid(np.arange(rows, dtype=np.uint64),
                         np.arange(col0, col0 + R, dtype=np.uint64), indexing="ij")
    u = rng.bits64(seed, tensor_id, rr, cc, rng.make_tag(stream, mode, rep), t)
    return rng.uniform_closed0(u).reshape(rows, R)


def cp_als(mttkrp, dims, R, iters, B0, C0):
    """CP-ALS with a fixed number of sweeps (Sec. 3.1 "Decompose").

    Each sweep updates modes 1, 2, 3 in order.  For mode n:
      M = MTTKRP_n, V = Hadamard product of the Gram matrices of the two other
      factors, U_n = M V^{-1}, lambda_f = ||U_n(:, f)||_2, U_n(:, f) /= lambda_f
      when lambda_f > 0.
    A is computed first from the initial B0, C0.
    `mttkrp(factors, mode)` supplies the tensor.
    Returns ([A, B, C], lam, pinv_count).
    """
    U = [np.zeros((dims[0], R)), np.array(B0, dtype=np.float64), np.array(C0, dtype=np.float64)]
    G = [None, U[1].T @ U[1], U[2].T @ U[2]]
    lam = np.ones(R)
    npinv = 0
    for _ in range(iters):
        for n in range(3):
            M = mttkrp(U, n)
            o1, o2 = [m for m in range(3) if m != n]
            V = G[o1] * G[o2]
            Un, used = solve_normal(M, V)
            npinv += int(used)
            Un, lam = normalize_columns(Un)
            U[n] = Un
            G[n] = Un.T @ Un
    return U, lam, npinv


def sort_by_weight(A, B, C, lam):
    """Order components by lambda descending; ties keep the lower index first."""
    order = np.argsort(-lam, kind="stable")
    return A[:, order], B[:, order], C[:, order], lam[order]


def fit_gram(normX2, A, B, C, lam, M3):
    """fit = 1 - ||X - Xhat||_F / ||X||_F (relative error of Sec. 4.2) via

    ||X - Xhat||^2 = ||X||^2 - 2 <X, Xhat> + ||Xhat||^2,
    ||Xhat||^2 = lam^T (A^T A * B^T B * C^T C) lam,
    <X, Xhat>  = sum_f lam_f sum_k C(k, f) M3(k, f),  M3 = X_(3) (B kr A).
    """
    H = (A.T @ A) * (B.T @ B) * (C.T @ C)
    xhat2 = float(lam @ H @ lam)
    inner = float(np.sum(lam[None, :] * C * M3))
    res2 = max(0.0, normX2 - 2.0 * inner + xhat2)
    return 1.0 - np.sqrt(res2) / np.sqrt(normX2)


def fit_explicit(X, A, B, C, lam):
    """1 - ||X - Xhat||_F / ||X||_F by forming Xhat (small tensors only)."""
    X = np.asarray(X, dtype=np.float64)
    Xh = reconstruct(A, B, C, lam)
    return 1.0 - np.linalg.norm((X - Xh).ravel()) / np.linalg.norm(X.ravel())


def fms(A1, B1, C1, lam1, A2, B2, C2, lam2):
    """Factor match score in [0, 1] after the best column permutation.

    Sec. 4.4 defines it as a penalised product of per-mode cosines; the
    printed formula also multiplies by 100 and sums, which contradicts the
    0..1 range stated in the text, so the score is averaged over R here.
    """
    from scipy.optimize import linear_sum_assignment
    R = A1.shape[1]
    cos = np.ones((R, R))
    for U, V in ((A1, A2), (B1, B2), (C1, C2)):
        Un, _ = normalize_columns(U)
        Vn, _ = normalize_columns(V)
        cos = cos * np.abs(Un.T @ Vn)
    rows, cols = linear_sum_assignment(cos, maximize=True)
    lam1 = np.abs(lam1 * np.linalg.norm(A1, axis=0) * np.linalg.norm(B1, axis=0)
                  * np.linalg.norm(C1, axis=0))
    lam2 = np.abs(lam2 * np.linalg.norm(A2, axis=0) * np.linalg.norm(B2, axis=0)
                  * np.linalg.norm(C2, axis=0))
    score = 0.0
    for r, c in zip(rows, cols):
        pen = 1.0 - abs(lam1[r] - lam2[c]) / max(lam1[r], lam2[c])
        score += pen * cos[r, c]
    return score / R


def corcondia(Z, A, B, C, lam):
    """Core consistency diagnostic (Sec. 3.2; Bro and Kiers) of the model
    (A, B, C, lam) of the dense tensor Z, in percent.

    The weights go into the third factor.  G = Z x1 pinv(A) x2 pinv(B)
    x3 pinv(C diag(lam)) is the least-squares Tucker core for the model's
    factors; the core of a perfect trilinear fit is superdiagonal with ones
    (T), and CC = 100 (1 - ||G - T||^2 / R).
    """
    Z = np.asarray(Z, dtype=np.float64)
    R = A.shape[1]
    Pa = np.linalg.pinv(A)
    Pb = np.linalg.pinv(B)
    Pc = np.linalg.pinv(C * np.asarray(lam)[None, :])
    G = np.einsum("ai,bj,ck,ijk->abc", Pa, Pb, Pc, Z, optimize=True)
    T = np.zeros((R, R, R))
    T[np.arange(R), np.arange(R), np.arange(R)] = 1.0
    return 100.0 * (1.0 - float(np.sum((G - T) ** 2)) / R)


def corcondia_coo(idx, vals, dims, A, B, C, lam):
    """The core consistency of corcondia() for a COO tensor: the same core
    G = Z x1 pinv(A) x2 pinv(B) x3 pinv(C diag(lam)), summed nonzero by
    nonzero, G(a, b, c) = sum over (x, y, z, v) of v Pa(a, x) Pb(b, y) Pc(c, z)
    (the zero entries add nothing; the sparse form the paper uses).  idx is
    (nnz, 3) int, vals (nnz,) float; dims only checks the coordinates."""
    idx = np.asarray(idx, dtype=np.int64).reshape(-1, 3)
    v = np.asarray(vals, dtype=np.float64)
    assert all(idx[:, m].max(initial=-1) < dims[m] for m in range(3))
    R = A.shape[1]
    Pa = np.linalg.pinv(A)
    Pb = np.linalg.pinv(B)
    Pc = np.linalg.pinv(C * np.asarray(lam)[None, :])
    G = np.einsum("e,ae,be,ce->abc", v, Pa[:, idx[:, 0]], Pb[:, idx[:, 1]], Pc[:, idx[:, 2]],
                  optimize=True)
    T = np.zeros((R, R, R))
    T[np.arange(R), np.arange(R), np.arange(R)] = 1.0
    return 100.0 * (1.0 - float(np.sum((G - T) ** 2)) / R)


def get_rank(Z, R, runs, threshold, iters, init):
    """GetRank (Sec. 3.2, Alg. 2) on the summary Z: a dense array, or a COO
    tensor given as (idx, vals, dims), whose CP-ALS runs over its entries
    and whose core consistency is summed over them (corcondia_coo).

    Every candidate rank i = 1..R gets `runs` CP-ALS runs (fixed `iters`
    sweeps) from the initial factors init(i, q) -> (B0, C0), q the run's
    index (i - 1) * runs + j; each run is scored by its core consistency.
    A core consistency of 100 is reached by every rank-1 model, so taking
    the single highest score would always return 1; the rank returned is
    the largest i whose best run reaches `threshold` (rank 1 always counts).
    Returns (R_new, (A, B, C), lam, cc) with the factors of the best run at
    R_new (the first of equal scores) and cc[i - 1][j] the scores.
    """
    if isinstance(Z, tuple):
        idx, vals, dims = Z

        def mtt(F, mode):
            return mttkrp_coo(idx, vals, F, mode, dims)

        def score_of(A, B, C, lam):
            return corcondia_coo(idx, vals, dims, A, B, C, lam)
    else:
        dims = Z.shape

        def mtt(F, mode):
            return mttkrp_dense(Z, F, mode)

        def score_of(A, B, C, lam):
            return corcondia(Z, A, B, C, lam)

    cc = []
    best = None
    for i in range(1, R + 1):
        row = []
        top = None  # (score, factors, lam) of the best run at rank i
        for j in range(runs):
            B0, C0 = init(i, (i - 1) * runs + j)
            (A, B, C), lam, _ = cp_als(mtt, dims, i, iters, B0, C0)
            score = score_of(A, B, C, lam)
            row.append(score)
            if top is None or score > top[0]:
                top = (score, (A, B, C), lam)
        cc.append(row)
        if i == 1 or top[0] >= threshold:
            best = (i, top[1], top[2])
    return best[0], best[1], best[2], cc
