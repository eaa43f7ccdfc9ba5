"""SamBaTen on a tensor of any order N >= 3, in plain FP64 (oracle; test
infrastructure).

Sec. 2 poses the problem for a third-order tensor whose third mode grows and
adds that the problem and the method carry over to any number of modes.  The
paper spells out only the third-order case, so the generalisation below is a
reading; at N = 3 every step is the third-order update of `sambaten.py`, and
the tests check that the two agree there.  Readings for N > 3:

* The last mode grows with the batches; every other mode is fixed.  A batch
  is K_new slices along the last mode.
* Measure of importance (Eq. 1) of index i of mode m: the sum of x^2 over all
  entries whose m-th index is i, in the exact integer form of the
  third-order case.  N_max, the most entries one index can collect, is the
  largest product of the other extents, the last one at its capacity.
* Every mode m has its own sampling factor s_m and is sampled n_m =
  ceil(D_m / s_m) times without replacement (last mode: among the K_old
  existing slices) by exponential keys from Philox counter
  (i, 0, tag(SAMPLE, m + 1, rep), t), as for three modes.
* The summary is X(S_0, ..., S_{N-2}, K_s u new).
* CP-ALS on a summary: modes 0, 1, ..., N-1 in turn; for mode n,
  U_n = MTTKRP_n V^-1 with V the Hadamard product of the Gram matrices of
  the N - 1 other factors; columns normalised after every mode.  U_1 ...
  U_{N-1} start U[0,1) from Philox tag(ALSINIT, m + 1, rep); U_0 is computed
  first.
* Matching: similarity S(f, g) = product over all N modes of |cosine|
  between the anchor rows of the current model and the summary factor (the
  last mode over its K_s rows); maximum-weight assignment; the sign of every
  fixed mode's matched column from that mode's cosine.
* New rows of the last factor: least squares against the Khatri-Rao product
  of the matched, sign-fixed fixed-mode factors rescaled to the anchor norms,
  divided by lambda; averaged over the valid repetitions in ascending order.
* Zero entries of every fixed-mode factor and of the last factor's anchor
  rows take the mean over the valid covering repetitions.
* lambda is kept.

Tensors are NumPy arrays of shape (D_0, ..., D_{N-1}); factor matrices are
row-major (rows x R).
"""

import numpy as np
from scipy.optimize import linear_sum_assignment

from . import cp, rng
from .sambaten import moi_scale, quantize_sq, sample_mode, sample_size, NumericError

_LETTERS = "abcdefghijklmnop"


# ----------------------------------------------------------------------------
# CP model of order N (Sec. 2.1 with N factors)
# ----------------------------------------------------------------------------

def mttkrp(X, factors, n):
    """M(i_n, r) = sum over all entries X(i_0, ..., i_{N-1}) times the
    product over m != n of U_m(i_m, r): the matricised tensor times the
    Khatri-Rao product of the other factors, written as one sum."""
    X = np.asarray(X, dtype=np.float64)
    N = X.ndim
    modes = _LETTERS[:N]
    ops = [X]
    subs = [modes]
    for m in range(N):
        if m != n:
            ops.append(np.asarray(factors[m], dtype=np.float64))
            subs.append(modes[m] + "z")
    return np.einsum(",".join(subs) + "->" + modes[n] + "z", *ops, optimize=True)


def reconstruct(factors, lam=None):
    """Full tensor of sum_r lam_r U_0(:, r) o ... o U_{N-1}(:, r)."""
    N = len(factors)
    R = factors[0].shape[1]
    lam = np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)
    modes = _LETTERS[:N]
    subs = ",".join(m + "z" for m in modes) + ",z->" + modes
    return np.einsum(subs, *factors, lam, optimize=True)


def moi(q):
    """Per-index sums of q over all other modes, one uint64 vector per mode."""
    q = np.asarray(q, dtype=np.uint64)
    N = q.ndim
    return [q.sum(axis=tuple(a for a in range(N) if a != m), dtype=np.uint64) for m in range(N)]


def cp_als(mttkrp_fn, dims, R, iters, U0):
    """CP-ALS with a fixed number of sweeps over modes 0..N-1 (Sec. 3.1
    "Decompose" for N factors).  U0[1:] are the initial factors (U0[0] is not
    read: mode 0 is computed first).  Returns (factors, lam, pinv_count)."""
    N = len(dims)
    U = [np.zeros((dims[0], R))] + [np.array(u, dtype=np.float64) for u in U0[1:]]
    G = [None] + [u.T @ u for u in U[1:]]
    lam = np.ones(R)
    npinv = 0
    for _ in range(iters):
        for n in range(N):
            M = mttkrp_fn(U, n)
            V = np.ones((R, R))
            for m in range(N):
                if m != n:
                    V = V * G[m]
            Un, used = cp.solve_normal(M, V)
            npinv += int(used)
            Un, lam = cp.normalize_columns(Un)
            U[n] = Un
            G[n] = Un.T @ Un
    return U, lam, npinv


def sort_by_weight(factors, lam):
    """Components ordered by lambda descending (ties keep the lower index)."""
    order = np.argsort(-lam, kind="stable")
    return [U[:, order] for U in factors], lam[order]


def fit_gram(normX2, factors, lam, M_last):
    """1 - ||X - Xhat|| / ||X|| from ||X||^2, the Gram matrices and the
    last-mode MTTKRP (the third-order expansion of Sec. 4.2 with N factors)."""
    R = len(lam)
    H = np.ones((R, R))
    for U in factors:
        H = H * (U.T @ U)
    xhat2 = float(lam @ H @ lam)
    inner = float(np.sum(lam[None, :] * factors[-1] * M_last))
    res2 = max(0.0, normX2 - 2.0 * inner + xhat2)
    return 1.0 - np.sqrt(res2) / np.sqrt(normX2)


# ----------------------------------------------------------------------------
# Matching (Sec. 3.1 "Project back", Lemma 1, over N modes)
# ----------------------------------------------------------------------------

def match(anchors, samples):
    """anchors[m]: rows of the current factor m at the sampled indices (the
    last mode: at K_s); samples[m]: the summary factor (the last mode: its
    K_s rows).  Returns (pi, signs, anchor_norms, S, cos) with signs and
    anchor_norms for the fixed modes 0..N-2."""
    N = len(anchors)
    cos = []
    for m in range(N):
        Ah, _ = cp.normalize_columns(anchors[m])
        Sh, _ = cp.normalize_columns(samples[m])
        cos.append(Ah.T @ Sh)
    R = cos[0].shape[0]
    S = np.ones((R, R))
    for m in range(N):
        S = S * np.abs(cos[m])
    rows, cols = linear_sum_assignment(S, maximize=True)
    pi = np.full(R, -1, dtype=np.int64)
    pi[rows] = cols
    signs, norms = [], []
    for m in range(N - 1):
        c = np.array([cos[m][f, pi[f]] if pi[f] >= 0 else 1.0 for f in range(R)])
        signs.append(np.where(c < 0, -1.0, 1.0))
        norms.append(np.sqrt(np.sum(anchors[m] * anchors[m], axis=0)))
    return pi, signs, norms, S, cos


# ----------------------------------------------------------------------------
# The tensor state and the update
# ----------------------------------------------------------------------------

class Config:
    """summary_bf16: the summaries are rounded to bfloat16 (nearest, ties to
    even) before their CP-ALS, as a path that stores them in BF16 does; every
    other step stays in FP64."""

    def __init__(self, rank, reps, als_iters, sample_factor, seed, order, tensor_id=0,
                 init_iters=100, k_capacity=None, summary_bf16=False):
        self.rank = int(rank)
        self.reps = int(reps)
        self.als_iters = int(als_iters)
        self.order = int(order)
        s = sample_factor
        self.s = (int(s),) * self.order if np.isscalar(s) else tuple(int(v) for v in s)
        assert len(self.s) == self.order
        self.seed = int(seed)
        self.tensor_id = int(tensor_id)
        self.init_iters = int(init_iters)
        self.k_capacity = k_capacity
        self.summary_bf16 = bool(summary_bf16)


class OracleTensorN:
    """Resident N-mode tensor + CP model + importance, updated batch by batch."""

    def __init__(self, cfg, X0, factors=None, lam=None, k_capacity=None):
        self.cfg = cfg
        X0 = np.asarray(X0)
        N = X0.ndim
        assert N == cfg.order and N >= 3
        self.N = N
        self.dims = list(X0.shape)
        self.X = np.asfortranarray(X0)
        self.t = 0
        kcap = k_capacity or cfg.k_capacity or self.dims[-1]
        cap = self.dims[:-1] + [int(kcap)]
        self.n_max = max(int(np.prod([cap[l] for l in range(N) if l != m])) for m in range(N))
        v = np.asarray(X0, dtype=np.float64)
        max_x2 = float(np.max(v * v)) if v.size else 0.0
        self.S = moi_scale(max_x2, self.n_max)
        q, ok = quantize_sq(self.X, self.S, self.n_max)
        if not ok:
            raise NumericError("initial tensor: non-finite value or MoI overflow")
        self.w = moi(q)
        if factors is None:
            self.U, self.lam = self.init_cp()
        else:
            self.U = [np.array(u, dtype=np.float64) for u in factors]
            self.lam = np.array(lam, dtype=np.float64)
        R = cfg.rank
        assert all(self.U[m].shape == (self.dims[m], R) for m in range(N))

    def init_cp(self):
        """CP-ALS on the whole initial tensor (problem statement of Sec. 2.2);
        U_1 ... U_{N-1} start U[0,1) from Philox tag(INIT, m + 1, 0)."""
        cfg = self.cfg
        R = cfg.rank
        U0 = [None] + [cp.als_init_factor(cfg.seed, cfg.tensor_id, rng.TAG_INIT, m + 1, 0, 0,
                                          self.dims[m], R) for m in range(1, self.N)]
        X = self.X
        U, lam, _ = cp_als(lambda F, n: mttkrp(X, F, n), self.dims, R, cfg.init_iters, U0)
        return sort_by_weight(U, lam)

    def update(self, Y, debug=False):
        """One batch of K_new last-mode slices (Algorithm 1 over N modes)."""
        cfg = self.cfg
        N, R = self.N, cfg.rank
        Y = np.asarray(Y)
        assert list(Y.shape[:-1]) == self.dims[:-1]
        Kn = Y.shape[-1]
        if Kn < 1:
            raise ValueError("empty batch")
        q, ok = quantize_sq(Y, self.S, self.n_max)
        if not ok:
            raise NumericError("batch: non-finite value or MoI overflow")
        Kold = self.dims[-1]
        XY = np.concatenate([self.X, Y], axis=N - 1)
        n = [sample_size(self.dims[m], cfg.s[m]) for m in range(N)]
        reps = []
        for rho in range(cfg.reps):
            Ss = [sample_mode(self.w[m], n[m], cfg.seed, cfg.tensor_id, m + 1, rho, self.t)
                  for m in range(N)]
            Ks = Ss[-1]
            Kp = np.concatenate([Ks, Kold + np.arange(Kn)])
            Z = np.asarray(XY[np.ix_(*(Ss[:-1] + [Kp]))], dtype=np.float64)
            if cfg.summary_bf16:
                Z = cp.round_bf16(Z)
            dims_s = list(Z.shape)
            U0 = [None] + [cp.als_init_factor(cfg.seed, cfg.tensor_id, rng.TAG_ALSINIT, m + 1,
                                              rho, self.t, dims_s[m], R) for m in range(1, N)]
            Up, lamp, npinv = cp_als(lambda F, m, Z=Z: mttkrp(Z, F, m), dims_s, R,
                                     cfg.als_iters, U0)
            n3 = len(Ks)
            anchors = [self.U[m][Ss[m]] for m in range(N - 1)] + [self.U[-1][Ks]]
            samples = Up[:-1] + [Up[-1][:n3]]
            pi, signs, norms, S, cos = match(anchors, samples)
            matched = pi >= 0
            valid = matched.copy()
            for m in range(N - 1):
                valid &= norms[m] > 0
            Ut = []
            for m in range(N - 1):
                Un, _ = cp.normalize_columns(Up[m])
                T = np.zeros((dims_s[m], R))
                T[:, matched] = Un[:, pi[matched]] * (signs[m] * norms[m])[None, matched]
                Ut.append(T)
            # least squares for every last-mode row of the summary
            G = np.ones((R, R))
            for m in range(N - 1):
                G = G * (Ut[m].T @ Ut[m])
            G[~matched, :] = 0.0
            G[:, ~matched] = 0.0
            G[~matched, ~matched] = 1.0
            Dm = mttkrp(Z, Ut + [None], N - 1)
            D, _ = cp.solve_normal(Dm, G)
            Ct = np.zeros_like(D)
            lz = self.lam > 0
            Ct[:, lz] = D[:, lz] / self.lam[lz]
            reps.append(dict(S=Ss, Up=Up, lamp=lamp, pi=pi, signs=signs, norms=norms, valid=valid,
                             Ut=Ut, Ct=Ct, Dm=Dm, npinv=npinv, Z=Z if debug else None))

        newU = [u.copy() for u in self.U]
        # zero entries of the fixed modes and of the last mode's anchor rows
        for m in range(N - 1):
            _zero_fill(newU[m], self.U[m], [(r["S"][m], r["Ut"][m], r["valid"]) for r in reps])
        _zero_fill(newU[-1], self.U[-1],
                   [(r["S"][-1], r["Ct"][:len(r["S"][-1])], r["valid"]) for r in reps])
        C_new = np.zeros((Kn, R))
        for f in range(R):
            acc = np.zeros(Kn)
            cnt = 0
            for r in reps:
                if r["valid"][f]:
                    acc = acc + r["Ct"][len(r["S"][-1]):, f]
                    cnt += 1
            if cnt:
                C_new[:, f] = acc / cnt
        self.U = newU[:-1] + [np.vstack([newU[-1], C_new])]
        self.X = np.asfortranarray(XY)
        dw = moi(q)
        self.w = [self.w[m] + dw[m] for m in range(N - 1)] + [np.concatenate([self.w[-1],
                                                                              dw[-1]])]
        self.dims[-1] = Kold + Kn
        self.t += 1
        if debug:
            return dict(reps=reps, C_new=C_new, n=n)
        return None

    def norm2(self):
        v = np.asarray(self.X, dtype=np.float64)
        return float(np.sum(v * v))

    def fit(self):
        M = mttkrp(self.X, self.U, self.N - 1)
        return fit_gram(self.norm2(), self.U, self.lam, M)

    def fit_explicit(self):
        X = np.asarray(self.X, dtype=np.float64)
        Xh = reconstruct(self.U, self.lam)
        return 1.0 - np.linalg.norm((X - Xh).ravel()) / np.linalg.norm(X.ravel())


def _zero_fill(out, cur, rep_rows):
    """out(i, f) = mean over the valid repetitions that sampled i of their
    row for i, wherever cur(i, f) == 0 exactly (Algorithm 1)."""
    R = cur.shape[1]
    for f in range(R):
        for i in np.nonzero(cur[:, f] == 0.0)[0]:
            acc, cnt = 0.0, 0
            for rows, U, valid in rep_rows:
                if not valid[f]:
                    continue
                p = np.searchsorted(rows, i)
                if p < len(rows) and rows[p] == i:
                    acc = acc + U[p, f]
                    cnt += 1
            if cnt:
                out[i, f] = acc / cnt

