"""The SamBaTen batch update in plain FP64 (oracle; test infrastructure).

Follows Algorithm 1 and the text of Sec. 3.1 step by step.  Where the paper
is silent or ambiguous the following readings are taken (all of them are
listed, with reasons, in the design notes of the repository):

* Measure of importance (Eq. 1) over the tensor *before* the update, computed
  once per batch (it does not depend on the repetition) and kept as exact
  integers: q(x) = floor(x*x * 2^S) summed in uint64, where the scale
  S = 58 - e2 - bitlen(N_max) is fixed at init from max x^2 = f * 2^e2
  (f in [0.5, 1)) of the initial tensor and N_max, the largest number of
  entries any index can collect at capacity.  An entry with
  q > floor(2^63 / N_max), or a non-finite entry, is a numeric error.
* Weighted sampling without replacement = successive sampling, realised with
  exponential keys (Efraimidis-Spirakis): kappa_i = E_i / double(w_i) with
  E_i = -ln(U_i) from Philox counter (i, 0, tag(SAMPLE, mode, rep), t);
  kappa = +inf for w_i = 0.  The n = ceil(N/s) smallest keys are chosen, ties
  by the smaller index, and returned in ascending index order.
* The summary is a plain restriction X(I_s, J_s, K_s u new), no re-weighting.
  Third-mode order: the sampled old slices ascending, then the new slices in
  arrival order.
* CP-ALS on each summary: fixed iterations, modes 1, 2, 3, U[0,1) initial
  B', C' from Philox (tag ALSINIT), Cholesky with a pseudo-inverse fallback,
  column normalisation after every mode (see cp.cp_als).
* Matching: anchors A(I_s), B(J_s), C(K_s) and the sample factors are column
  normalised (C' over its anchor rows only); similarity S(f, g) is the product
  over the three modes of |cosine|; the permutation is a maximum-weight
  perfect assignment; signs come from the A and B cosines.
* The new rows of C are the least-squares solution against the matched,
  sign-fixed sample factors rescaled to the units of A(I_s), B(J_s), divided
  by lambda; they are averaged over the valid repetitions in ascending order.
* Zero entries of A, B and the anchor rows of C are replaced by the mean over
  the valid covering repetitions, after all repetitions (order free).
* lambda is kept unchanged by default.  With lambda_avg (the last step of
  Algorithm 1 read literally), lambda becomes the average of its previous
  value and the new one, the new one being the mean over the repetitions
  valid for the component (with a non-zero C(K_s) column) of the summary's
  matched weight in the current model's units:
  lambda'_pi(f) ||C'(anchor rows, pi(f))|| / (||A(I_s, f)|| ||B(J_s, f)||
  ||C(K_s, f)||), which equals lambda_f when the summary recovers the
  restriction of the current model exactly.
* Persistent summaries (optional; Sec. 3.1 assumes summaries of the tensor
  already exist when a batch arrives): the sampled I_s, J_s, K_s of an update are kept for the
  following ones (redrawn every summary_refresh updates), so a summary is
  X(I_s, J_s, K_s u new) with the same anchors each time, and its CP-ALS
  starts from the previous summary factors (B', and C' on the K_s rows; the
  rows of the new slices drawn U[0,1) as usual).
* GetRank (Sec. 3.2, optional): per summary, R_new = the largest candidate
  rank whose best CP run reaches the core-consistency threshold (see
  cp.get_rank); the summary's factors are that run's.  The R_new sample
  components are matched to R_new of the R current ones (maximum-weight
  assignment); a current component left without a partner contributes
  nothing from that repetition (its new rows are averaged over the
  repetitions that matched it, zero if none did).
"""

import math

import numpy as np
from scipy.optimize import linear_sum_assignment

from . import cp, rng

DENSE, COO = 0, 1


# ----------------------------------------------------------------------------
# Measure of importance (Eq. 1), exact integer form
# ----------------------------------------------------------------------------

def moi_scale(max_x2, n_max):
    """Fixed-point scale S such that N_max entries of size max_x2 sum < 2^58."""
    if not (max_x2 > 0.0):
        return 32
    _, e2 = math.frexp(max_x2)
    return 58 - e2 - int(n_max).bit_length()


def quantize_sq(x, S, n_max):
    """q = floor(x*x * 2^S) as uint64; returns (q, ok)."""
    x = np.asarray(x, dtype=np.float64)
    x2s = (x * x) * math.ldexp(1.0, S)
    ok = bool(np.all(x2s < 2.0 ** 63))
    if not ok:
        return None, False
    q = np.floor(x2s).astype(np.uint64)
    qmax = np.uint64((1 << 63) // int(n_max))
    if np.any(q > qmax):
        return None, False
    return q, True


def moi_dense(q):
    """Per-index sums of q over the other two modes (Eq. 1 and its mode-2/3
    analogues).  q has shape (I, J, K)."""
    return (q.sum(axis=(1, 2), dtype=np.uint64), q.sum(axis=(0, 2), dtype=np.uint64),
            q.sum(axis=(0, 1), dtype=np.uint64))


def moi_coo(idx, q, dims):
    out = []
    for m in range(3):
        w = np.zeros(dims[m], dtype=np.uint64)
        np.add.at(w, idx[:, m], q)
        out.append(w)
    return out


# ----------------------------------------------------------------------------
# Weighted sampling without replacement (Sec. 3.1 "Sample", Algorithm 1)
# ----------------------------------------------------------------------------

def sample_keys(w, seed, tensor_id, mode, rep, t):
    """kappa_i = -ln(U_i) / double(w_i); +inf where w_i == 0."""
    N = len(w)
    u = rng.bits64(seed, tensor_id, np.arange(N, dtype=np.uint64), 0,
                   rng.make_tag(rng.TAG_SAMPLE, mode, rep), t)
    E = rng.exp_variate(u)
    wd = np.asarray(w, dtype=np.uint64).astype(np.float64)
    kappa = np.full(N, np.inf)
    pos = wd > 0
    kappa[pos] = E[pos] / wd[pos]
    return kappa


def sample_mode(w, n, seed, tensor_id, mode, rep, t):
    """The n indices with the smallest keys (ties: smaller index), ascending."""
    kappa = sample_keys(w, seed, tensor_id, mode, rep, t)
    order = np.argsort(kappa, kind="stable")
    return np.sort(order[:n]).astype(np.int64)


def sample_size(N, s):
    """n = ceil(N / s), at least 1 and at most N."""
    return max(1, min(N, -(-N // s)))


# ----------------------------------------------------------------------------
# Matching (Sec. 3.1 "Project back", Lemma 1)
# ----------------------------------------------------------------------------

def match(A_anchor, B_anchor, C_anchor, Ap, Bp, Cp_anchor):
    """Returns (pi, sigA, sigB, nA, nB, S, cosA, cosB).

    pi[f] is the sample column matched to current column f, -1 when the
    sample has fewer columns than the model and f is left over.
    """
    Ah, nA = cp.normalize_columns(A_anchor)
    Bh, nB = cp.normalize_columns(B_anchor)
    Ch, _ = cp.normalize_columns(C_anchor)
    Apn, _ = cp.normalize_columns(Ap)
    Bpn, _ = cp.normalize_columns(Bp)
    Cpn, _ = cp.normalize_columns(Cp_anchor)
    cosA = Ah.T @ Apn
    cosB = Bh.T @ Bpn
    cosC = Ch.T @ Cpn
    S = np.abs(cosA) * np.abs(cosB) * np.abs(cosC)
    rows, cols = linear_sum_assignment(S, maximize=True)
    pi = np.full(S.shape[0], -1, dtype=np.int64)  # -1: no sample column left (R_new < R)
    pi[rows] = cols
    R = S.shape[0]
    sA = np.array([cosA[f, pi[f]] if pi[f] >= 0 else 1.0 for f in range(R)])
    sB = np.array([cosB[f, pi[f]] if pi[f] >= 0 else 1.0 for f in range(R)])
    sigA = np.where(sA < 0, -1.0, 1.0)
    sigB = np.where(sB < 0, -1.0, 1.0)
    return pi, sigA, sigB, nA, nB, S, cosA, cosB


# ----------------------------------------------------------------------------
# The tensor state and the update
# ----------------------------------------------------------------------------

class Config:
    def __init__(self, rank, reps, als_iters, sample_factor, seed, tensor_id=0,
                 init_iters=100, k_capacity=None, nnz_capacity=None, summary_bf16=False,
                 getrank_runs=0, getrank_threshold=90.0, persist_summaries=False,
                 summary_refresh=0, workers=1, lambda_avg=False):
        self.rank = int(rank)
        self.reps = int(reps)
        self.als_iters = int(als_iters)
        s = sample_factor
        self.s = (int(s),) * 3 if np.isscalar(s) else tuple(int(v) for v in s)
        self.seed = int(seed)
        self.tensor_id = int(tensor_id)
        self.init_iters = int(init_iters)
        self.k_capacity = k_capacity
        self.nnz_capacity = nnz_capacity
        # dense summaries stored as bfloat16 (rounded to nearest even) before
        # the decomposition and the row solve; everything else stays FP64
        self.summary_bf16 = bool(summary_bf16)
        # GetRank (Sec. 3.2, Alg. 2) on every summary when getrank_runs > 0
        self.getrank_runs = int(getrank_runs)
        self.getrank_threshold = float(getrank_threshold)
        # persistent summaries (Sec. 3.1 assumes summaries of the tensor exist
        # before the update): the sampled indices are kept from one update to the next
        # (redrawn every summary_refresh updates, never when 0) and the summary
        # CP-ALS starts from the previous summary factors
        self.persist_summaries = bool(persist_summaries)
        self.summary_refresh = int(summary_refresh)
        # host threads for the independent repetitions and for blocks of slices
        # (scheduling only: every result is the same for any count)
        self.workers = max(1, int(workers))
        # the paper's lambda update (Alg. 1, last step) instead of keeping lambda
        self.lambda_avg = bool(lambda_avg)
        if self.persist_summaries and self.getrank_runs > 0:
            raise ValueError("persistent summaries and GetRank do not combine")


class NumericError(ValueError):
    pass


def _map_ordered(fn, items, workers):
    """[fn(x) for x in items], on `workers` threads when workers > 1 (each
    call's BLAS then runs on one thread); the results keep the items' order."""
    items = list(items)
    if workers <= 1 or len(items) <= 1:
        return [fn(x) for x in items]
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1, user_api="blas"):
        with ThreadPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(fn, items))


def _slice_blocks(X, block=32):
    """Consecutive blocks of frontal slices of a dense (I, J, K) array (views)."""
    for k0 in range(0, X.shape[2], block):
        yield X[:, :, k0:k0 + block]


class OracleTensor:
    """Resident tensor + CP model + sampling state, updated batch by batch."""

    def __init__(self, cfg, fmt, dims, X0=None, coo0=None, factors=None, k_capacity=None):
        self.cfg = cfg
        self.fmt = fmt
        I, J, K0 = (int(d) for d in dims)
        self.I, self.J, self.K = I, J, K0
        self.t = 0
        self.kept = None  # persistent summaries: per repetition (Is, Js, Ks, B', C')
        kcap = k_capacity or cfg.k_capacity or K0
        if fmt == DENSE:
            X0 = np.asarray(X0)
            assert X0.shape == (I, J, K0)
            self.X = np.asfortranarray(X0)
            n_max = max(J * kcap, I * kcap, I * J)
            max_x2 = max([0.0] + _map_ordered(
                lambda blk: float(np.max(np.asarray(blk, dtype=np.float64) ** 2)),
                _slice_blocks(self.X), cfg.workers))
        else:
            idx, vals = coo0
            self.idx = np.asarray(idx, dtype=np.int64).reshape(-1, 3)
            self.vals = np.asarray(vals)
            n_max = max(J * kcap, I * kcap, I * J)
            if cfg.nnz_capacity:
                n_max = min(n_max, int(cfg.nnz_capacity))
            v64 = np.asarray(self.vals, dtype=np.float64)
            max_x2 = float(np.max(v64 * v64)) if v64.size else 0.0
        self.n_max = n_max
        self.S = moi_scale(max_x2, n_max)
        if fmt == DENSE:
            w, ok = self._moi_dense(self.X)
        else:
            q, ok = self._quant_all(self.vals)
            w = self._moi(q, (I, J, K0), None) if ok else None
        if not ok:
            raise NumericError("initial tensor: non-finite value or MoI overflow")
        self.w = w
        R = cfg.rank
        if factors is None:
            A, B, C, lam = self.init_cp()
        else:
            A, B, C, lam = (np.array(f, dtype=np.float64) for f in factors)
        self.A, self.B, self.C, self.lam = A, B, C, lam
        assert self.A.shape == (I, R) and self.B.shape == (J, R) and self.C.shape == (K0, R)

    # -- helpers ---------------------------------------------------------------
    def _data_values(self):
        return self.X if self.fmt == DENSE else self.vals

    def _quant_all(self, x):
        return quantize_sq(x, self.S, self.n_max)

    def _moi_dense(self, X):
        """Eq. 1 of a dense block, taken over blocks of slices (the sums are
        exact integers, so the blocking does not change them).  Returns
        ([w1, w2, w3], ok)."""
        def block_moi(blk):
            q, ok = self._quant_all(blk)
            return moi_dense(q) if ok else None

        parts = _map_ordered(block_moi, _slice_blocks(X), self.cfg.workers)
        if any(p is None for p in parts):
            return None, False
        w1 = np.zeros(X.shape[0], dtype=np.uint64)
        w2 = np.zeros(X.shape[1], dtype=np.uint64)
        for d1, d2, _ in parts:
            w1 += d1
            w2 += d2
        w3 = np.concatenate([p[2] for p in parts]) if parts else np.zeros(0, dtype=np.uint64)
        return [w1, w2, w3], True

    def _moi(self, q, dims, idx):
        if self.fmt == DENSE:
            return list(moi_dense(q))
        return moi_coo(idx if idx is not None else self.idx, q, dims)

    def mttkrp_full(self, factors, mode):
        if self.fmt == DENSE:
            return cp.mttkrp_dense(self.X, factors, mode)
        return cp.mttkrp_coo(self.idx, self.vals, factors, mode, (self.I, self.J, self.K))

    # -- initial decomposition (problem statement of Sec. 2.2) ------------------
    def init_cp(self):
        cfg = self.cfg
        R = cfg.rank
        B0 = cp.als_init_factor(cfg.seed, cfg.tensor_id, rng.TAG_INIT, 2, 0, 0, self.J, R)
        C0 = cp.als_init_factor(cfg.seed, cfg.tensor_id, rng.TAG_INIT, 3, 0, 0, self.K, R)
        (A, B, C), lam, _ = cp.cp_als(self.mttkrp_full, (self.I, self.J, self.K), R,
                                       cfg.init_iters, B0, C0)
        return cp.sort_by_weight(A, B, C, lam)

    # -- the update (Algorithm 1) -------------------------------------------------
    def update(self, Y=None, coo=None, debug=False):
        cfg = self.cfg
        I, J, Kold, R = self.I, self.J, self.K, cfg.rank
        if self.fmt == DENSE:
            Y = np.asarray(Y)
            assert Y.shape[0] == I and Y.shape[1] == J
            Kn = Y.shape[2]
            dw, ok = self._moi_dense(Y)
        else:
            yidx, yvals, Kn = coo
            yidx = np.asarray(yidx, dtype=np.int64).reshape(-1, 3)
            yvals = np.asarray(yvals)
            q, ok = self._quant_all(yvals)
        if Kn < 1:
            raise ValueError("empty batch")
        if not ok:
            raise NumericError("batch: non-finite value or MoI overflow")

        # Summaries are taken from X u Y: append first, sample from the old part.
        if self.fmt == DENSE:
            # column-major like the stored tensor (the unfoldings are views of it)
            XY = np.empty((I, J, Kold + Kn), dtype=np.result_type(self.X, Y), order="F")
            XY[:, :, :Kold] = self.X
            XY[:, :, Kold:] = Y
        else:
            shifted = yidx.copy()
            shifted[:, 2] += Kold
            XYidx = np.concatenate([self.idx, shifted])
            XYvals = np.concatenate([self.vals, yvals])

        n = [sample_size(I, cfg.s[0]), sample_size(J, cfg.s[1]), sample_size(Kold, cfg.s[2])]
        reuse = (cfg.persist_summaries and self.kept is not None and
                 not (cfg.summary_refresh > 0 and self.t % cfg.summary_refresh == 0))
        def one_rep(rho):
            if reuse:
                Is, Js, Ks = self.kept[rho][:3]
            else:
                Is = sample_mode(self.w[0], n[0], cfg.seed, cfg.tensor_id, 1, rho, self.t)
                Js = sample_mode(self.w[1], n[1], cfg.seed, cfg.tensor_id, 2, rho, self.t)
                Ks = sample_mode(self.w[2], n[2], cfg.seed, cfg.tensor_id, 3, rho, self.t)
            Kp = np.concatenate([Ks, Kold + np.arange(Kn)])
            dims_s = (len(Is), len(Js), len(Kp))
            if self.fmt == DENSE:
                Z = np.asfortranarray(XY[np.ix_(Is, Js, Kp)], dtype=np.float64)
                if cfg.summary_bf16:
                    Z = cp.round_bf16(Z)

                def mtt(F, mode, Z=Z):
                    return cp.mttkrp_dense(Z, F, mode)
            else:
                Zidx, Zval = self._gather_coo(XYidx, XYvals, Is, Js, Kp, I, J, Kold + Kn)

                def mtt(F, mode, Zidx=Zidx, Zval=Zval, dims_s=dims_s):
                    return cp.mttkrp_coo(Zidx, Zval, F, mode, dims_s)
            Rn, cc = R, None
            if cfg.getrank_runs > 0:
                # GetRank (Sec. 3.2) before the decomposition: the summary's
                # rank R_new <= R and the best of its CP runs at that rank
                # (a sparse summary's runs and scores go over its entries)
                if self.fmt != DENSE:
                    Z = (Zidx, Zval, dims_s)

                def init(i, q, rho=rho, dims_s=dims_s):
                    return tuple(cp.als_init_factor(cfg.seed, cfg.tensor_id, rng.TAG_GETRANK,
                                                    m, rho, self.t, dims_s[m - 1], i,
                                                    col0=32 * q) for m in (2, 3))
                Rn, (Ap, Bp, Cp), lamp, cc = cp.get_rank(Z, R, cfg.getrank_runs,
                                                         cfg.getrank_threshold, cfg.als_iters,
                                                         init)
                npinv = 0
            else:
                # Decompose (Sec. 3.1), B' and C' drawn U[0,1), A' computed first;
                # with kept summaries B' and the K_s rows of C' start from the
                # previous summary factors (warm start)
                B0 = cp.als_init_factor(cfg.seed, cfg.tensor_id, rng.TAG_ALSINIT, 2, rho, self.t,
                                        dims_s[1], R)
                C0 = cp.als_init_factor(cfg.seed, cfg.tensor_id, rng.TAG_ALSINIT, 3, rho, self.t,
                                        dims_s[2], R)
                if reuse:
                    B0 = self.kept[rho][3].copy()
                    C0[:len(Ks)] = self.kept[rho][4]
                (Ap, Bp, Cp), lamp, npinv = cp.cp_als(mtt, dims_s, R, cfg.als_iters, B0, C0)
            # Normalise + match (Sec. 3.1 "Project back", Lemma 1); with
            # R_new < R only R_new of the current components find a partner.
            n3 = len(Ks)
            pi, sigA, sigB, nA, nB, S, cosA, cosB = match(
                self.A[Is], self.B[Js], self.C[Ks], Ap, Bp, Cp[:n3])
            matched = pi >= 0
            valid = (nA > 0) & (nB > 0) & matched
            Apn, _ = cp.normalize_columns(Ap)
            Bpn, _ = cp.normalize_columns(Bp)
            At = np.zeros((len(Is), R))
            Bt = np.zeros((len(Js), R))
            At[:, matched] = Apn[:, pi[matched]] * (sigA * nA)[None, matched]
            Bt[:, matched] = Bpn[:, pi[matched]] * (sigB * nB)[None, matched]
            # Row least squares for every third-mode row of the summary; an
            # unmatched component gets a unit diagonal (its rows come out zero).
            G = (At.T @ At) * (Bt.T @ Bt)
            G[~matched, :] = 0.0
            G[:, ~matched] = 0.0
            G[~matched, ~matched] = 1.0
            Dm = mtt([At, Bt, None], 2)
            D, _ = cp.solve_normal(Dm, G)
            Ct = np.zeros_like(D)
            lz = self.lam > 0
            Ct[:, lz] = D[:, lz] / self.lam[lz]
            # the summary's weights of the matched components in the current units
            nC = np.linalg.norm(self.C[Ks], axis=0)
            ncp = np.linalg.norm(Cp[:n3], axis=0)
            lhat = np.full(R, np.nan)
            for f in range(R):
                if valid[f] and nC[f] > 0:
                    lhat[f] = lamp[pi[f]] * ncp[pi[f]] / (nA[f] * nB[f] * nC[f])
            return dict(Is=Is, Js=Js, Ks=Ks, Ap=Ap, Bp=Bp, Cp=Cp, lamp=lamp, pi=pi, lhat=lhat,
                        sigA=sigA, sigB=sigB, nA=nA, nB=nB, S=S, valid=valid, At=At,
                        Bt=Bt, Ct=Ct, Dm=Dm, npinv=npinv, Rnew=Rn, cc=cc)

        # the repetitions are independent (Sec. 3.1: no synchronisation between
        # them); with workers > 1 they run concurrently, collected in order
        reps = _map_ordered(one_rep, range(cfg.reps), cfg.workers)

        A_new, B_new, C_old = self.A.copy(), self.B.copy(), self.C.copy()
        # Zero-entry update over the sampled rows (Algorithm 1), order free.
        self._zero_fill(A_new, self.A, [(r["Is"], r["At"], r["valid"]) for r in reps])
        self._zero_fill(B_new, self.B, [(r["Js"], r["Bt"], r["valid"]) for r in reps])
        self._zero_fill(C_old, self.C, [(r["Ks"], r["Ct"][:len(r["Ks"])], r["valid"])
                                        for r in reps])
        # Average of the new rows over the valid repetitions, ascending order.
        C_new = np.zeros((Kn, R))
        for f in range(R):
            acc = np.zeros(Kn)
            cnt = 0
            for r in reps:
                if r["valid"][f]:
                    acc = acc + r["Ct"][len(r["Ks"]):, f]
                    cnt += 1
            if cnt:
                C_new[:, f] = acc / cnt

        # lambda: kept, or the average of the previous and the new value
        lam_new = self.lam.copy()
        if cfg.lambda_avg:
            for f in range(R):
                acc, cnt = 0.0, 0
                for r in reps:
                    if not np.isnan(r["lhat"][f]):
                        acc = acc + r["lhat"][f]
                        cnt += 1
                if cnt:
                    lam_new[f] = 0.5 * (self.lam[f] + acc / cnt)

        # Commit the state.
        if cfg.persist_summaries:
            self.kept = [(r["Is"], r["Js"], r["Ks"], r["Bp"].copy(), r["Cp"][:len(r["Ks"])].copy())
                         for r in reps]
        self.A, self.B = A_new, B_new
        self.C = np.vstack([C_old, C_new])
        self.lam = lam_new
        if self.fmt == DENSE:
            self.X = XY
            self.w = [self.w[0] + dw[0], self.w[1] + dw[1], np.concatenate([self.w[2], dw[2]])]
        else:
            self.idx, self.vals = XYidx, XYvals
            dw = moi_coo(yidx, q, (I, J, Kn))
            self.w = [self.w[0] + dw[0], self.w[1] + dw[1], np.concatenate([self.w[2], dw[2]])]
        self.K = Kold + Kn
        self.t += 1
        if debug:
            return dict(reps=reps, C_new=C_new, n=n)
        return None

    @staticmethod
    def _gather_coo(idx, vals, Is, Js, Kp, I, J, K):
        posI = np.full(I, -1, dtype=np.int64)
        posJ = np.full(J, -1, dtype=np.int64)
        posK = np.full(K, -1, dtype=np.int64)
        posI[Is] = np.arange(len(Is))
        posJ[Js] = np.arange(len(Js))
        posK[Kp] = np.arange(len(Kp))
        a, b, c = posI[idx[:, 0]], posJ[idx[:, 1]], posK[idx[:, 2]]
        keep = (a >= 0) & (b >= 0) & (c >= 0)
        return np.stack([a[keep], b[keep], c[keep]], axis=1), np.asarray(vals)[keep]

    @staticmethod
    def _zero_fill(out, cur, rep_rows):
        R = cur.shape[1]
        for f in range(R):
            zero_rows = np.nonzero(cur[:, f] == 0.0)[0]
            if zero_rows.size == 0:
                continue
            for i in zero_rows:
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

    # -- fit (Sec. 4.2 relative error) ---------------------------------------------
    def norm2(self):
        if self.fmt == DENSE:
            def block_sum(blk):
                v = np.asarray(blk, dtype=np.float64)
                return float(np.sum(v * v))
            total = 0.0
            for part in _map_ordered(block_sum, _slice_blocks(self.X), self.cfg.workers):
                total += part
            return total
        v = np.asarray(self.vals, dtype=np.float64)
        return float(np.sum(v * v))

    def fit(self):
        if self.fmt == DENSE:
            # X_(3) (B kr A) row by row of slices: row k depends on slice k only
            KR = cp.khatri_rao(self.B, self.A)
            M3 = np.vstack(_map_ordered(
                lambda blk: cp.unfold(np.asarray(blk, dtype=np.float64), 2) @ KR,
                _slice_blocks(self.X, 64), self.cfg.workers))
        else:
            M3 = self.mttkrp_full([self.A, self.B, self.C], 2)
        return cp.fit_gram(self.norm2(), self.A, self.B, self.C, self.lam, M3)

    def fit_explicit(self):
        assert self.fmt == DENSE
        return cp.fit_explicit(self.X, self.A, self.B, self.C, self.lam)
