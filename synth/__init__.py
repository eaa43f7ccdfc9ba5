"""Seeded synthetic inputs shaped like the paper's workloads (Sec. 4.1.1).

This module only produces data: a low-rank CP model with U[0,1) factors plus
Gaussian noise at a given fraction of the tensor norm (dense), or nonzeros
drawn from a nonnegative CP model with Zipf row popularity (sparse COO).  It
contains none of the update's arithmetic.  The oracle and the HIP path both
consume its outputs bit for bit.

Randomness comes from NumPy's Philox bit generator keyed by SeedSequence
(seed, stream, block), so a slice block can be regenerated on its own.
"""

import numpy as np

STREAM_FACTOR = 11
STREAM_NOISE = 12
STREAM_SPARSE = 13
STREAM_ARRIVAL = 14


def _gen(seed, stream, block=0):
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, stream, block])))


class DenseCP:
    """X = sum_r A(:,r) o B(:,r) o C(:,r) + N(0, sigma^2), factors U[0,1) (or
    N(0,1) with factors="normal").

    sigma = noise * ||X_clean||_F / sqrt(I*J*K), with ||X_clean||^2 taken in
    closed form from the factor Gram matrices, so the noise is `noise` of the
    tensor norm in expectation and slices can be produced in any order.
    """

    def __init__(self, I, J, K, R, seed, noise=0.01, dtype=np.float32, factors="uniform"):
        self.I, self.J, self.K, self.R = int(I), int(J), int(K), int(R)
        self.seed, self.noise, self.dtype = int(seed), float(noise), np.dtype(dtype)
        g = _gen(seed, STREAM_FACTOR)
        # factor entries U[0,1) (nonnegative, nearly collinear columns) or N(0,1)
        # (nearly orthogonal columns)
        draw = g.random if factors == "uniform" else g.standard_normal
        self.A = draw((self.I, self.R))
        self.B = draw((self.J, self.R))
        self.C = draw((self.K, self.R))
        H = (self.A.T @ self.A) * (self.B.T @ self.B) * (self.C.T @ self.C)
        self.clean_norm2 = float(H.sum())
        self.sigma = self.noise * np.sqrt(self.clean_norm2 / (self.I * self.J * self.K))

    def slices(self, k0, k1, block=256):
        """Frontal slices k0..k1-1 as an (I, J, k1-k0) Fortran-ordered array."""
        out = np.empty((self.I, self.J, k1 - k0), dtype=self.dtype, order="F")
        for b0 in range(k0, k1, block):
            b1 = min(k1, b0 + block)
            # X_(3) rows = C (B kr A)^T for the block, built slice by slice in FP64
            for k in range(b0, b1):
                S = (self.A * self.C[k][None, :]) @ self.B.T
                if self.noise > 0:
                    S = S + self.sigma * _gen(self.seed, STREAM_NOISE, k).standard_normal(
                        (self.I, self.J))
                out[:, :, k - k0] = S.astype(self.dtype)
        return out

    def fill_slices_kji(self, out, k0, k1, workers=16):
        """Slices k0..k1-1 written into out[k - k0] as (J, I) arrays: the
        memory of `out` (shape (k1 - k0, J, I), C order) is then the
        column-major layout of the (I, J, k1 - k0) tensor.  Values are those of
        slices(); slices are produced in parallel."""
        from concurrent.futures import ThreadPoolExecutor

        def one(k):
            S = (self.A * self.C[k][None, :]) @ self.B.T
            if self.noise > 0:
                S = S + self.sigma * _gen(self.seed, STREAM_NOISE, k).standard_normal(
                    (self.I, self.J))
            out[k - k0] = S.astype(self.dtype).T

        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(k0, k1)))
        return out

    def fill_device(self, torch, out, k0=0, block=64):
        """The same model with noise drawn on the GPU, for tensors too large to
        generate on the host: out (a CUDA tensor of shape (k1 - k0, J, I), the
        column-major layout of the (I, J, k1 - k0) tensor) receives slices
        k0..k1-1, each B diag(C(k, :)) A^T in FP64 plus sigma times standard
        normals from a CUDA generator seeded per block of slices, rounded to
        out's dtype.  The noise differs from slices(); both sides of a
        comparison must read the bytes written here (copy them to the host for
        the oracle)."""
        dev = out.device
        At = torch.from_numpy(np.ascontiguousarray(self.A.T)).to(dev)     # (R, I)
        Bd = torch.from_numpy(self.B).to(dev)                              # (J, R)
        Cd = torch.from_numpy(self.C).to(dev)                              # (K, R)
        k1 = k0 + out.shape[0]
        gen = torch.Generator(device=dev)
        for b0 in range(k0, k1, block):
            b1 = min(k1, b0 + block)
            blk = torch.matmul(Bd[None, :, :] * Cd[b0:b1, None, :], At)   # (k, J, I)
            if self.noise > 0:
                gen.manual_seed((self.seed * 1000003 + STREAM_NOISE) * 1000003 + b0)
                blk += self.sigma * torch.randn(blk.shape, generator=gen, device=dev,
                                                dtype=torch.float64)
            out[b0 - k0:b1 - k0] = blk.to(out.dtype)
        return out

    def true_model(self):
        """Ground-truth factors normalised to unit columns, weights in lambda,
        ordered by lambda descending."""
        nA = np.linalg.norm(self.A, axis=0)
        nB = np.linalg.norm(self.B, axis=0)
        nC0 = np.linalg.norm(self.C, axis=0)
        lam = nA * nB * nC0
        order = np.argsort(-lam, kind="stable")
        return (self.A[:, order] / nA[order], self.B[:, order] / nB[order],
                self.C[:, order] / nC0[order], lam[order])

    def true_model_prefix(self, K0):
        """Unit A, B; C restricted to the first K0 slices, in the same units
        as true_model() (so C rows of later slices continue the same scale)."""
        A, B, C, lam = self.true_model()
        return A, B, C[:K0].copy(), lam


class SparseSupportCP:
    """A sparse tensor of exact low rank: X = sum_r A(:,r) o B(:,r) o C(:,r)
    with factor entries 0.5 + U[0,1) on about `support` of the rows of each
    column and zero elsewhere, so X is zero outside the union of R boxes.  The
    nonzeros of slice k get N(0, noise^2) from the noise stream of block k (in
    the order of (i, j)) and are rounded to FP32.  For rank estimation on
    sparse data (the rank is R wherever the boxes are sampled); built box by
    box, so large tensors need no dense array.
    """

    def __init__(self, I, J, K, R, seed, support=0.4, noise=1e-3):
        self.I, self.J, self.K, self.R = int(I), int(J), int(K), int(R)
        self.seed, self.noise = int(seed), float(noise)
        g = _gen(seed, STREAM_FACTOR)
        self.F = [np.where(g.random((n, self.R)) < support, 0.5 + g.random((n, self.R)), 0.0)
                  for n in (self.I, self.J, self.K)]

    def entries(self, k0, k1):
        """The nonzeros of slices k0..k1-1: coordinates (third one relative to
        k0), ordered by k, then i, then j, and FP32 values."""
        A, B, C = self.F
        I, J = self.I, self.J
        keys, vals = [], []
        for r in range(self.R):
            ia = np.nonzero(A[:, r])[0]
            jb = np.nonzero(B[:, r])[0]
            kc = np.nonzero(C[k0:k1, r])[0]
            if len(ia) == 0 or len(jb) == 0 or len(kc) == 0:
                continue
            key = (kc[:, None, None] * I + ia[None, :, None]) * J + jb[None, None, :]
            v = C[k0 + kc, r][:, None, None] * A[ia, r][None, :, None] * B[jb, r][None, None, :]
            keys.append(key.ravel())
            vals.append(v.ravel())
        if not keys:
            return np.zeros((0, 3), dtype=np.int64), np.zeros(0, dtype=np.float32)
        key, inv = np.unique(np.concatenate(keys), return_inverse=True)
        x = np.bincount(inv, weights=np.concatenate(vals), minlength=len(key))
        k = key // (I * J)
        i = (key // J) % I
        j = key % J
        if self.noise > 0:
            bounds = np.searchsorted(k, np.arange(k1 - k0 + 1))
            for kk in range(k1 - k0):
                a, b = bounds[kk], bounds[kk + 1]
                if b > a:
                    x[a:b] += self.noise * _gen(self.seed, STREAM_NOISE, k0 + kk).standard_normal(
                        b - a)
        return np.stack([i, j, k], axis=1), x.astype(np.float32)

    def dense(self, k0, k1):
        """Slices k0..k1-1 as an FP64 array holding the values of entries()."""
        idx, v = self.entries(k0, k1)
        X = np.zeros((self.I, self.J, k1 - k0))
        X[tuple(idx.T)] = v
        return X


class SparseCP:
    """COO nonzeros drawn from a nonnegative rank-R model.

    For component r: Zipf(zipf) popularity over a random permutation of the
    indices of modes 1 and 2, and a U[0,1) profile over mode 3.  A nonzero
    picks a component uniformly, then i, j, k from the three profiles;
    duplicates on the key (i*J + j)*K + k are dropped and the draw topped up
    until nnz distinct coordinates exist.  The value is the model entry
    sum_r lam_r a_r(i) b_r(j) c_r(k) (scaled to mean ~1) plus N(0, sigma^2),
    sigma = noise * ||v_clean|| / sqrt(nnz).
    """

    def __init__(self, I, J, K, R, seed, zipf=1.1, noise=0.01):
        self.I, self.J, self.K, self.R = int(I), int(J), int(K), int(R)
        self.seed, self.zipf, self.noise = int(seed), float(zipf), float(noise)
        g = _gen(seed, STREAM_FACTOR)
        self.pa = np.empty((self.R, self.I))
        self.pb = np.empty((self.R, self.J))
        for r in range(self.R):
            self.pa[r, g.permutation(self.I)] = (1.0 + np.arange(self.I)) ** (-self.zipf)
            self.pb[r, g.permutation(self.J)] = (1.0 + np.arange(self.J)) ** (-self.zipf)
        self.pc = g.random((self.R, self.K))
        self.pa /= self.pa.sum(axis=1, keepdims=True)
        self.pb /= self.pb.sum(axis=1, keepdims=True)
        self.pc /= self.pc.sum(axis=1, keepdims=True)
        self.scale = 1.0

    def _model_values(self, idx):
        v = np.zeros(idx.shape[0])
        for r in range(self.R):
            v += self.pa[r, idx[:, 0]] * self.pb[r, idx[:, 1]] * self.pc[r, idx[:, 2]]
        return v

    def slices(self, k0, k1, nnz, block_id=0):
        """About `nnz` distinct nonzeros with k in [k0, k1); returns
        (idx (nnz,3) int32 with k relative to k0, vals float32)."""
        g = _gen(self.seed, STREAM_SPARSE, block_id)
        keys = np.empty(0, dtype=np.int64)
        span = k1 - k0
        pc = self.pc[:, k0:k1]
        pc = pc / pc.sum(axis=1, keepdims=True)
        cum_a = np.cumsum(self.pa, axis=1)
        cum_b = np.cumsum(self.pb, axis=1)
        cum_c = np.cumsum(pc, axis=1)
        while keys.size < nnz:
            m = int((nnz - keys.size) * 1.2) + 16
            comp = g.integers(0, self.R, size=m)
            ii = np.empty(m, dtype=np.int64)
            jj = np.empty(m, dtype=np.int64)
            kk = np.empty(m, dtype=np.int64)
            for r in range(self.R):
                sel = comp == r
                cnt = int(sel.sum())
                if cnt == 0:
                    continue
                ii[sel] = np.minimum(np.searchsorted(cum_a[r], g.random(cnt) * cum_a[r, -1]),
                                     self.I - 1)
                jj[sel] = np.minimum(np.searchsorted(cum_b[r], g.random(cnt) * cum_b[r, -1]),
                                     self.J - 1)
                kk[sel] = np.minimum(np.searchsorted(cum_c[r], g.random(cnt) * cum_c[r, -1]),
                                     span - 1)
            new = (ii * self.J + jj) * span + kk
            keys = np.unique(np.concatenate([keys, new]))
        keys = keys[g.permutation(keys.size)[:nnz]]
        keys.sort()
        kk = keys % span
        ij = keys // span
        jj = ij % self.J
        ii = ij // self.J
        idx = np.stack([ii, jj, kk], axis=1)
        full = idx.copy()
        full[:, 2] += k0
        v = self._model_values(full)
        mean = v.mean() if v.size else 1.0
        self.last_mean = float(mean)
        v = v / mean
        if self.noise > 0 and v.size:
            sigma = self.noise * np.linalg.norm(v) / np.sqrt(v.size)
            v = v + sigma * g.standard_normal(v.size)
        return idx.astype(np.int32), v.astype(np.float32)


class SparseCPN:
    """The N-mode analogue of SparseCP: for component r, Zipf(zipf) popularity
    over a random permutation of the indices of every leading mode and a
    U[0,1) profile over the last mode; a nonzero picks a component uniformly,
    then one index per mode from the profiles; duplicates are dropped and the
    draw topped up.  The value is sum_r prod_m P_m(i_m, r) scaled to mean 1,
    plus N(0, sigma^2) with sigma = noise * ||v|| / sqrt(nnz)."""

    def __init__(self, dims, R, seed, zipf=1.1, noise=0.01):
        self.dims = tuple(int(d) for d in dims)
        self.R, self.seed, self.zipf, self.noise = int(R), int(seed), float(zipf), float(noise)
        g = _gen(seed, STREAM_FACTOR)
        self.P = []
        for d in self.dims[:-1]:
            P = np.empty((self.R, d))
            for r in range(self.R):
                P[r, g.permutation(d)] = (1.0 + np.arange(d)) ** (-self.zipf)
            self.P.append(P / P.sum(axis=1, keepdims=True))
        pc = g.random((self.R, self.dims[-1]))
        self.P.append(pc / pc.sum(axis=1, keepdims=True))

    def slices(self, k0, k1, nnz, block_id=0):
        """About `nnz` distinct nonzeros with last index in [k0, k1): a list of
        N int32 coordinate arrays (the last relative to k0) ordered by the
        linear index with the first mode slowest, and FP32 values."""
        g = _gen(self.seed, STREAM_SPARSE, block_id)
        ext = list(self.dims[:-1]) + [k1 - k0]
        N = len(ext)
        prof = [P for P in self.P[:-1]] + [self.P[-1][:, k0:k1]]
        cums = [np.cumsum(P, axis=1) for P in prof]
        keys = np.empty(0, dtype=np.int64)
        while keys.size < nnz:
            m = int((nnz - keys.size) * 1.2) + 16
            comp = g.integers(0, self.R, size=m)
            co = [np.empty(m, dtype=np.int64) for _ in range(N)]
            for r in range(self.R):
                sel = comp == r
                cnt = int(sel.sum())
                if cnt == 0:
                    continue
                for q in range(N):
                    c = cums[q][r]
                    co[q][sel] = np.minimum(np.searchsorted(c, g.random(cnt) * c[-1]), ext[q] - 1)
            new = co[0]
            for q in range(1, N):
                new = new * ext[q] + co[q]
            keys = np.unique(np.concatenate([keys, new]))
        keys = keys[g.permutation(keys.size)[:nnz]]
        keys.sort()
        cols = []
        rest = keys
        for q in range(N - 1, -1, -1):
            cols.append(rest % ext[q])
            rest = rest // ext[q]
        cols = cols[::-1]
        v = np.zeros(keys.size)
        for r in range(self.R):
            t = np.ones(keys.size)
            for q in range(N):
                t = t * prof[q][r, cols[q]]
            v += t
        v = v / (v.mean() if v.size else 1.0)
        if self.noise > 0 and v.size:
            v = v + self.noise * np.linalg.norm(v) / np.sqrt(v.size) * g.standard_normal(v.size)
        return [c.astype(np.int32) for c in cols], v.astype(np.float32)


def sparse_model(gen, K0, mean):
    """Factors of a SparseCP block whose values were divided by `mean`: unit
    columns A, B, C (C over the first K0 slices) and lambda, in SparseCP's
    component order."""
    A, B, C = gen.pa.T.copy(), gen.pb.T.copy(), gen.pc.T[:K0].copy()
    nA, nB, nC = (np.linalg.norm(M, axis=0) for M in (A, B, C))
    return A / nA, B / nB, C / nC, nA * nB * nC / mean


def poisson_arrivals(n, rate, seed):
    """Arrival times (s) of a Poisson process with `rate` requests per second."""
    g = _gen(seed, STREAM_ARRIVAL)
    return np.cumsum(g.exponential(1.0 / rate, size=n))


class DenseCPN:
    """The N-mode analogue of DenseCP: X = sum_r U_0(:,r) o ... o U_{N-1}(:,r)
    + N(0, sigma^2), factors U[0,1), the last mode the one that grows.

    Slices along the last mode are produced in any order; sigma = noise *
    ||X_clean||_F / sqrt(#entries) with ||X_clean||^2 in closed form.
    """

    def __init__(self, dims, R, seed, noise=0.01, dtype=np.float32):
        self.dims = tuple(int(d) for d in dims)
        self.R, self.seed, self.noise = int(R), int(seed), float(noise)
        self.dtype = np.dtype(dtype)
        g = _gen(seed, STREAM_FACTOR)
        self.U = [g.random((d, self.R)) for d in self.dims]
        H = np.ones((self.R, self.R))
        for U in self.U:
            H = H * (U.T @ U)
        self.clean_norm2 = float(H.sum())
        self.sigma = self.noise * np.sqrt(self.clean_norm2 / float(np.prod(self.dims)))

    def slices(self, k0, k1):
        """Last-mode slices k0..k1-1 as a Fortran-ordered array of shape
        dims[:-1] + (k1 - k0,)."""
        lead = self.dims[:-1]
        # Khatri-Rao rows of the leading modes, the first mode fastest
        K = np.ones((1, self.R))
        for U in self.U[:-1]:  # row a * P + p: the new mode slowest
            K = (U[:, None, :] * K[None, :, :]).reshape(-1, self.R)
        out = np.empty(lead + (k1 - k0,), dtype=self.dtype, order="F")
        n_lead = int(np.prod(lead))
        for k in range(k0, k1):
            v = K @ self.U[-1][k]
            if self.noise > 0:
                v = v + self.sigma * _gen(self.seed, STREAM_NOISE, k).standard_normal(n_lead)
            out[..., k - k0] = v.reshape(lead, order="F").astype(self.dtype)
        return out

    def true_model(self):
        """Unit-column factors and lambda, ordered by lambda descending."""
        norms = [np.linalg.norm(U, axis=0) for U in self.U]
        lam = np.prod(norms, axis=0)
        order = np.argsort(-lam, kind="stable")
        return [U[:, order] / n[order] for U, n in zip(self.U, norms)], lam[order]

    def true_model_prefix(self, K0):
        """true_model() with the last factor cut to its first K0 rows."""
        Us, lam = self.true_model()
        return Us[:-1] + [Us[-1][:K0].copy()], lam
