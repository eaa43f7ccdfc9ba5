"""Parity of the HIP sparse (COO) update path with the CPU FP64 oracle."""

import numpy as np
import pytest

import synth
from oracle import cp
from oracle import sambaten as osb
from parity import assert_close

# FP32 summaries and products against the FP64 oracle: factor entries within
# 1e-3 of the entry plus 1e-3 of the column's largest entry (the fit bar of
# 1e-3 carried to the factors), sampled indices and matchings exact
RT, AT = 1e-3, 1e-3

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def sparse_case(I, J, K0, Kn, batches, R, nnz0, nnz_b, seed):
    gen = synth.SparseCP(I, J, K0 + batches * Kn, R, seed=seed)
    idx0, v0 = gen.slices(0, K0, nnz0, block_id=0)
    bat = [gen.slices(K0 + b * Kn, K0 + (b + 1) * Kn, nnz_b, block_id=b + 1)
           for b in range(batches)]
    return idx0, v0, bat


def run_coo_pair(lib, I, J, K0, Kn, batches, R, reps, iters, s, seed, nnz0, nnz_b,
                 persist=False):
    torch = _torch()
    idx0, v0, bat = sparse_case(I, J, K0, Kn, batches, R, nnz0, nnz_b, seed)
    g = np.random.default_rng(seed)
    A0, B0, C0 = g.random((I, R)), g.random((J, R)), g.random((K0, R))
    nA, nB, nC = (np.linalg.norm(M, axis=0) for M in (A0, B0, C0))
    model = (A0 / nA, B0 / nB, C0 / nC, nA * nB * nC)
    kcap = K0 + batches * Kn
    ocfg = osb.Config(rank=R, reps=reps, als_iters=iters, sample_factor=s, seed=seed,
                      k_capacity=kcap, nnz_capacity=nnz0 + batches * nnz_b,
                      persist_summaries=persist)
    ora = osb.OracleTensor(ocfg, osb.COO, (I, J, K0), coo0=(idx0, v0), factors=model)
    cfg = lib.make_config(R, reps, iters, s, seed, fmt=lib.SBT_COO, precision=lib.SBT_P_F32,
                          k_capacity=kcap, max_batch=Kn, nnz_capacity=nnz0 + batches * nnz_b,
                          persist_summaries=persist)
    cols, vd = lib.coo_to_device(idx0, v0)
    gpu = lib.Tensor.init_coo(cfg, cols, vd, len(v0), I, J, K0, model)
    ds = []
    for yidx, yv in bat:
        d = ora.update(coo=(yidx, yv, Kn), debug=True)
        bcols, bv = lib.coo_to_device(yidx, yv)
        gpu.update_batch_coo(bcols, bv, len(yv), Kn)
        torch.cuda.synchronize()
        ds.append(d)
    return ora, gpu, ds


def check_coo_update(lib, ora, gpu, d, reps, K0, n1):
    for rho in range(reps):
        for mode, key in enumerate(("Is", "Js", "Ks")):
            np.testing.assert_array_equal(gpu.last_sample(rho, mode), d["reps"][rho][key],
                                          err_msg=f"rep {rho} mode {mode}")
        r = d["reps"][rho]
        np.testing.assert_array_equal(gpu.last_rep(rho, lib.SBT_REP_PI, 1)[0], r["pi"])
        assert_close(gpu.last_rep(rho, lib.SBT_REP_AP, n1), r["Ap"], RT, AT, f"A' rep {rho}")
        assert_close(gpu.last_rep(rho, lib.SBT_REP_CT, len(r["Ct"])), r["Ct"], RT, AT,
                     f"C~ rep {rho}")
    A, B, C, lam = gpu.get_factors()
    assert_close(C[K0:], ora.C[K0:], RT, AT, "new rows of C")
    assert_close(A, ora.A, RT, AT, "A")
    assert abs(gpu.fit() - ora.fit()) < 1e-3


def test_coo_update_matches_oracle(lib):
    reps = 4
    ora, gpu, ds = run_coo_pair(lib, 80, 70, 40, 10, 2, 3, reps, 15, 2, 21, 6000, 1500)
    check_coo_update(lib, ora, gpu, ds[-1], reps, 40, 40)
    assert gpu.shape()[2] == 60


def test_coo_ten_updates_track_the_oracle(lib):
    # Alg. 1 applied ten times over sparse batches: samples, matchings and the
    # last update's intermediates as above, the whole model at the end
    reps = 4
    ora, gpu, ds = run_coo_pair(lib, 60, 50, 30, 5, 10, 3, reps, 12, 2, 73, 4000, 700)
    check_coo_update(lib, ora, gpu, ds[-1], reps, 30, 30)
    A, B, C, lam = gpu.get_factors()
    assert_close(B, ora.B, RT, AT, "B")
    assert_close(C, ora.C, RT, AT, "C")
    assert gpu.batch_counter() == 10
    assert gpu.shape()[2] == 80


@pytest.mark.parametrize("I,J,K0,R,nnz0,nnz_b", [
    (80, 70, 40, 20, 6000, 1500),    # rank above 16: 32-float factor rows, 8 lanes per entry
    (60, 50, 40, 3, 50000, 6000),    # about 200 summary entries per row: a wavefront per unit
    # rank 10 (12 padded columns, the sparse workload's kernels) and rank 6 (8 columns):
    # about 50 summary entries per row of modes 1 and 2 (32 lanes per unit) and about 250
    # per row of mode 3 (64 lanes per unit)
    (200, 200, 20, 10, 40000, 20000),
    (200, 200, 20, 6, 40000, 20000),
])
def test_coo_update_unit_shapes(lib, I, J, K0, R, nnz0, nnz_b):
    reps = 3
    ora, gpu, ds = run_coo_pair(lib, I, J, K0, 10, 1, R, reps, 10, 2, 23, nnz0, nnz_b)
    check_coo_update(lib, ora, gpu, ds[-1], reps, K0, -(-I // 2))


def _coo_tensor(g, n1, n2, n3, nnz, heavy_row):
    """Distinct random coordinates, one row of mode 1 holding about 1500 entries
    (three work units of 512), FP32 values."""
    keys = g.choice(n1 * n2 * n3, size=nnz, replace=False)
    a, rest = keys % n1, keys // n1
    b, c = rest % n2, rest // n2
    hk = g.choice(n2 * n3, size=min(1500, n2 * n3), replace=False)
    a = np.concatenate([a, np.full(hk.size, heavy_row)])
    b = np.concatenate([b, hk % n2])
    c = np.concatenate([c, hk // n2])
    idx = np.unique(np.stack([a, b, c], axis=1), axis=0)
    idx = idx[g.permutation(len(idx))]
    v = (g.random(len(idx)) + 0.1).astype(np.float32)
    return idx.astype(np.int32), v


@pytest.mark.parametrize("R", [3, 6, 10, 20])
@pytest.mark.parametrize("lanes", [0, 32, 64])
def test_coo_mttkrp_relative_error(lib, R, lanes):
    # the sparse MTTKRP kernels of the update (ordering, work units, unit
    # kernel with 32 or 64 lanes, in-order sum of the unit partials) on one
    # COO tensor, every mode, against the oracle's entry-by-entry MTTKRP:
    # FP32 relative error <= 1e-5
    torch = _torch()
    g = np.random.default_rng(500 + R + lanes)
    n1, n2, n3 = 70, 55, 41
    idx, v = _coo_tensor(g, n1, n2, n3, 30000, heavy_row=7)
    U = [g.random((n, R)) for n in (n1, n2, n3)]
    cols, vd = lib.coo_to_device(idx, v)
    Ud = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in U]
    for mode in range(3):
        out = torch.zeros(((n1, n2, n3)[mode], R), dtype=torch.float64, device="cuda")
        lib.mttkrp_coo(cols, vd, len(v), n1, n2, n3, R, Ud[0], Ud[1], Ud[2], mode, out,
                       lanes=lanes)
        torch.cuda.synchronize()
        ref = cp.mttkrp_coo(idx.astype(np.int64), v.astype(np.float64), U, mode, (n1, n2, n3))
        got = out.cpu().numpy()
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert rel <= 1e-5, (mode, rel)
        assert_close(got, ref, 1e-5, 1e-6, f"mode {mode}")


def test_coo_mttkrp_empty_and_single_entry(lib):
    torch = _torch()
    R = 4
    U = [np.arange(n * R, dtype=np.float64).reshape(n, R) / 7.0 for n in (3, 4, 5)]
    Ud = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in U]
    for idx, v in ((np.zeros((0, 3), np.int32), np.zeros(0, np.float32)),
                   (np.array([[2, 3, 4]], np.int32), np.array([1.5], np.float32))):
        cols, vd = lib.coo_to_device(idx, v) if len(v) else (
            tuple(torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(3)),
            torch.zeros(1, dtype=torch.float32, device="cuda"))
        for mode in range(3):
            out = torch.full(((3, 4, 5)[mode], R), 7.0, dtype=torch.float64, device="cuda")
            lib.mttkrp_coo(cols, vd, len(v), 3, 4, 5, R, Ud[0], Ud[1], Ud[2], mode, out)
            torch.cuda.synchronize()
            ref = cp.mttkrp_coo(idx.astype(np.int64), v.astype(np.float64), U, mode, (3, 4, 5))
            np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-6, atol=0)


def test_sampler_at_sparse_workload_size(lib):
    # the sampler at the sparse workload's population (N = 1e5 per mode,
    # n = 1e4 drawn): about 30% of the mode-1 indices have no entry (weight 0),
    # the weights are small integer multiples of one value, so many are tied;
    # mode 2 has only 5000 indices of positive weight, fewer than the 1e4
    # drawn, so the rest are taken from the zero weights in index order.
    # Bit-exact against the oracle's sampler on the same weights.
    torch = _torch()
    g = np.random.default_rng(77)
    I = J = 100_000
    K0, Kn, R, reps, s = 1000, 10, 2, 3, 10
    nnz0 = 300_000
    live_i = g.choice(I, size=70_000, replace=False)
    live_j = g.choice(J, size=5_000, replace=False)
    keys = np.unique(live_i[g.integers(0, live_i.size, nnz0)].astype(np.int64) * J * K0
                     + live_j[g.integers(0, live_j.size, nnz0)].astype(np.int64) * K0
                     + g.integers(0, K0, nnz0))
    idx0 = np.stack([keys // (J * K0), (keys // K0) % J, keys % K0], axis=1)
    v0 = np.ones(len(keys), dtype=np.float32)
    nb = 2000
    bidx = np.stack([live_i[g.integers(0, live_i.size, nb)], live_j[g.integers(0, live_j.size, nb)],
                     g.integers(0, Kn, nb)], axis=1)
    bidx = np.unique(bidx, axis=0)
    bv = np.ones(len(bidx), dtype=np.float32)
    A0, B0, C0 = g.random((I, R)), g.random((J, R)), g.random((K0, R))
    nA, nB, nC = (np.linalg.norm(M, axis=0) for M in (A0, B0, C0))
    model = (A0 / nA, B0 / nB, C0 / nC, nA * nB * nC)
    ocfg = osb.Config(rank=R, reps=reps, als_iters=2, sample_factor=s, seed=77,
                      k_capacity=K0 + Kn, nnz_capacity=len(v0) + len(bv))
    ora = osb.OracleTensor(ocfg, osb.COO, (I, J, K0), coo0=(idx0, v0), factors=model)
    w = ora.w
    assert np.sum(w[0] == 0) >= 25_000 and np.sum(w[1] > 0) == 5_000
    assert len(np.unique(w[0])) < 100  # heavily tied weights
    cfg = lib.make_config(R, reps, 2, s, 77, fmt=lib.SBT_COO, precision=lib.SBT_P_F32,
                          k_capacity=K0 + Kn, max_batch=Kn, nnz_capacity=len(v0) + len(bv))
    cols, vd = lib.coo_to_device(idx0, v0)
    gpu = lib.Tensor.init_coo(cfg, cols, vd, len(v0), I, J, K0, model)
    d = ora.update(coo=(bidx, bv, Kn), debug=True)
    bcols, bvd = lib.coo_to_device(bidx, bv)
    gpu.update_batch_coo(bcols, bvd, len(bv), Kn)
    torch.cuda.synchronize()
    for rho in range(reps):
        for mode, key in enumerate(("Is", "Js", "Ks")):
            got = gpu.last_sample(rho, mode)
            want = d["reps"][rho][key]
            assert len(want) == (10_000, 10_000, 100)[mode]
            np.testing.assert_array_equal(got, want, err_msg=f"rep {rho} mode {mode}")
        Js = d["reps"][rho]["Js"]
        assert np.sum(w[1][Js] > 0) == 5_000
        # the zero-weight part of J_s is the smallest zero-weight indices
        zeros = np.nonzero(w[1] == 0)[0][:5_000]
        np.testing.assert_array_equal(np.sort(Js[w[1][Js] == 0]), zeros)


def test_coo_persistent_summaries(lib):
    reps = 3
    ora, gpu, ds = run_coo_pair(lib, 80, 70, 40, 10, 3, 3, reps, 12, 2, 25, 6000, 1500,
                                persist=True)
    for rho in range(reps):
        for mode, key in enumerate(("Is", "Js", "Ks")):
            np.testing.assert_array_equal(ds[-1]["reps"][rho][key], ds[0]["reps"][rho][key])
    check_coo_update(lib, ora, gpu, ds[-1], reps, 40, 40)


def test_coo_fit_matches_oracle_after_init(lib):
    torch = _torch()
    idx0, v0, _ = sparse_case(50, 40, 30, 5, 1, 2, 2000, 100, 5)
    g = np.random.default_rng(5)
    R = 2
    A0, B0, C0 = g.random((50, R)), g.random((40, R)), g.random((30, R))
    model = (A0, B0, C0, np.ones(R))
    ocfg = osb.Config(rank=R, reps=2, als_iters=3, sample_factor=2, seed=5, k_capacity=35,
                      nnz_capacity=2100)
    ora = osb.OracleTensor(ocfg, osb.COO, (50, 40, 30), coo0=(idx0, v0), factors=model)
    cfg = lib.make_config(R, 2, 3, 2, 5, fmt=lib.SBT_COO, k_capacity=35, max_batch=5,
                          nnz_capacity=2100)
    cols, vd = lib.coo_to_device(idx0, v0)
    gpu = lib.Tensor.init_coo(cfg, cols, vd, len(v0), 50, 40, 30, model)
    torch.cuda.synchronize()
    assert abs(gpu.fit() - ora.fit()) < 1e-9


def test_coo_rejects_out_of_range_batch(lib):
    torch = _torch()
    idx0, v0, bat = sparse_case(30, 30, 20, 5, 1, 2, 800, 200, 6)
    R = 2
    g = np.random.default_rng(6)
    model = (g.random((30, R)), g.random((30, R)), g.random((20, R)), np.ones(R))
    cfg = lib.make_config(R, 2, 3, 2, 6, fmt=lib.SBT_COO, k_capacity=25, max_batch=5,
                          nnz_capacity=1000)
    cols, vd = lib.coo_to_device(idx0, v0)
    gpu = lib.Tensor.init_coo(cfg, cols, vd, len(v0), 30, 30, 20, model)
    yidx, yv = bat[0]
    bad = yidx.copy()
    bad[3, 2] = 5  # k outside the batch
    bcols, bv = lib.coo_to_device(bad, yv)
    assert gpu.try_update_batch_coo(bcols, bv, len(yv), 5) == lib.SBT_E_SHAPE
    yv2 = yv.copy()
    yv2[0] = np.nan
    bcols, bv = lib.coo_to_device(yidx, yv2)
    assert gpu.try_update_batch_coo(bcols, bv, len(yv), 5) == lib.SBT_E_NUMERIC
    assert gpu.shape()[2] == 20 and gpu.batch_counter() == 0
    bcols, bv = lib.coo_to_device(yidx, yv)
    gpu.update_batch_coo(bcols, bv, len(yv), 5)
    torch.cuda.synchronize()
    assert gpu.shape()[2] == 25 and gpu.batch_counter() == 1


def test_coo_and_dense_storage_agree(lib):
    # the same tensor stored densely and as COO gives the same samples and update
    torch = _torch()
    I, J, K0, Kn, R, reps = 24, 20, 16, 4, 2, 3
    gen = synth.DenseCP(I, J, K0 + Kn, R, seed=8, dtype=np.float32)
    X = gen.slices(0, K0 + Kn)
    X[np.random.default_rng(8).random(X.shape) < 0.4] = 0.0
    model = gen.true_model_prefix(K0)
    cfg_d = lib.make_config(R, reps, 10, 2, 8, precision=lib.SBT_P_F32, k_capacity=K0 + Kn,
                            max_batch=Kn)
    gd = lib.Tensor.init_dense(cfg_d, lib.dense_to_device(X[:, :, :K0], np.float32), I, J, K0,
                               factors=model)
    nnz_all = int((X != 0).sum())
    cfg_c = lib.make_config(R, reps, 10, 2, 8, fmt=lib.SBT_COO, k_capacity=K0 + Kn,
                            max_batch=Kn, nnz_capacity=nnz_all)
    X0 = X[:, :, :K0]
    idx0 = np.argwhere(X0 != 0)
    cols, vd = lib.coo_to_device(idx0, X0[X0 != 0])
    gc = lib.Tensor.init_coo(cfg_c, cols, vd, len(idx0), I, J, K0, model)
    Y = X[:, :, K0:]
    yidx = np.argwhere(Y != 0)
    gd.update_batch_dense(lib.dense_to_device(Y, np.float32), Kn)
    bcols, bv = lib.coo_to_device(yidx, Y[Y != 0])
    gc.update_batch_coo(bcols, bv, len(yidx), Kn)
    torch.cuda.synchronize()
    for rho in range(reps):
        for mode in range(3):
            np.testing.assert_array_equal(gd.last_sample(rho, mode), gc.last_sample(rho, mode))
    Cd = gd.get_factors()[2]
    Cc = gc.get_factors()[2]
    np.testing.assert_allclose(Cc, Cd, rtol=1e-4, atol=1e-6)
    assert abs(gd.fit() - gc.fit()) < 1e-6


def test_coo_and_dense_persistent_summaries_agree(lib):
    # persistent summaries over four batches: the COO summaries keep their old
    # part and scan only each batch, the dense ones keep theirs in place; both
    # hold the same entries, so the updates agree at FP32 rounding level
    torch = _torch()
    I, J, K0, Kn, R, reps, nb = 26, 22, 18, 3, 2, 3, 4
    gen = synth.DenseCP(I, J, K0 + nb * Kn, R, seed=9, dtype=np.float32)
    X = gen.slices(0, K0 + nb * Kn)
    X[np.random.default_rng(9).random(X.shape) < 0.4] = 0.0
    model = gen.true_model_prefix(K0)
    kcap = K0 + nb * Kn
    cfg_d = lib.make_config(R, reps, 10, 2, 9, precision=lib.SBT_P_F32, k_capacity=kcap,
                            max_batch=Kn, persist_summaries=True)
    gd = lib.Tensor.init_dense(cfg_d, lib.dense_to_device(X[:, :, :K0], np.float32), I, J, K0,
                               factors=model)
    nnz_all = int((X != 0).sum())
    cfg_c = lib.make_config(R, reps, 10, 2, 9, fmt=lib.SBT_COO, k_capacity=kcap, max_batch=Kn,
                            nnz_capacity=nnz_all, persist_summaries=True)
    X0 = X[:, :, :K0]
    idx0 = np.argwhere(X0 != 0)
    cols, vd = lib.coo_to_device(idx0, X0[X0 != 0])
    gc = lib.Tensor.init_coo(cfg_c, cols, vd, len(idx0), I, J, K0, model)
    for b in range(nb):
        Y = X[:, :, K0 + b * Kn:K0 + (b + 1) * Kn]
        yidx = np.argwhere(Y != 0)
        gd.update_batch_dense(lib.dense_to_device(Y, np.float32), Kn)
        bcols, bv = lib.coo_to_device(yidx, Y[Y != 0])
        gc.update_batch_coo(bcols, bv, len(yidx), Kn)
        torch.cuda.synchronize()
        for rho in range(reps):
            for mode in range(3):
                np.testing.assert_array_equal(gd.last_sample(rho, mode),
                                              gc.last_sample(rho, mode))
        Cd = gd.get_factors()[2]
        Cc = gc.get_factors()[2]
        np.testing.assert_allclose(Cc, Cd, rtol=1e-4, atol=1e-6, err_msg=f"batch {b}")
    assert abs(gd.fit() - gc.fit()) < 1e-6


def test_coo_persistent_summaries_outgrowing_their_allocation(lib):
    # persistent COO summaries whose second batch is twenty times the first:
    # the summaries no longer fit what the first update allocated, so that
    # update rebuilds them from the store; the third keeps its old part again.
    # Dense storage of the same tensor is the reference at every step.
    torch = _torch()
    I, J, K0, R, reps = 40, 40, 20, 2, 3
    sizes = [1, 20, 3]
    Kall = K0 + sum(sizes)
    gen = synth.DenseCP(I, J, Kall, R, seed=11, dtype=np.float32)
    X = gen.slices(0, Kall)
    X[np.random.default_rng(11).random(X.shape) < 0.4] = 0.0
    model = gen.true_model_prefix(K0)
    cfg_d = lib.make_config(R, reps, 8, 2, 11, precision=lib.SBT_P_F32, k_capacity=Kall,
                            max_batch=max(sizes), persist_summaries=True)
    gd = lib.Tensor.init_dense(cfg_d, lib.dense_to_device(X[:, :, :K0], np.float32), I, J, K0,
                               factors=model)
    cfg_c = lib.make_config(R, reps, 8, 2, 11, fmt=lib.SBT_COO, k_capacity=Kall,
                            max_batch=max(sizes), nnz_capacity=int((X != 0).sum()),
                            persist_summaries=True)
    X0 = X[:, :, :K0]
    idx0 = np.argwhere(X0 != 0)
    cols, vd = lib.coo_to_device(idx0, X0[X0 != 0])
    gc = lib.Tensor.init_coo(cfg_c, cols, vd, len(idx0), I, J, K0, model)
    k = K0
    for b, kn in enumerate(sizes):
        Y = X[:, :, k:k + kn]
        k += kn
        yidx = np.argwhere(Y != 0)
        gd.update_batch_dense(lib.dense_to_device(Y, np.float32), kn)
        bcols, bv = lib.coo_to_device(yidx, Y[Y != 0])
        gc.update_batch_coo(bcols, bv, len(yidx), kn)
        torch.cuda.synchronize()
        np.testing.assert_allclose(gc.get_factors()[2], gd.get_factors()[2], rtol=1e-4,
                                   atol=1e-6, err_msg=f"batch {b}")
    assert abs(gd.fit() - gc.fit()) < 1e-6


@pytest.mark.parametrize("I,J,K0,R,nnz0,iters", [(80, 70, 40, 4, 6000, 25),
                                                 (300, 260, 90, 10, 40000, 15)])
def test_coo_initial_cp_als_matches_oracle(lib, I, J, K0, R, nnz0, iters):
    # no factors given: the initial decomposition is CP-ALS on the whole COO tensor
    # (the initial-stream U[0,1) start, init_iters sweeps, components by lambda);
    # FP32 sparse products against the oracle's FP64 CP-ALS of the same entries
    torch = _torch()
    gen = synth.SparseCP(I, J, K0 + 5, R, seed=91 + R)
    idx0, v0 = gen.slices(0, K0, nnz0, block_id=0)
    ocfg = osb.Config(rank=R, reps=2, als_iters=5, sample_factor=2, seed=91, k_capacity=K0 + 5,
                      nnz_capacity=nnz0 + 2000, init_iters=iters)
    ora = osb.OracleTensor(ocfg, osb.COO, (I, J, K0), coo0=(idx0, v0))
    cfg = lib.make_config(R, 2, 5, 2, 91, fmt=lib.SBT_COO, precision=lib.SBT_P_F32,
                          k_capacity=K0 + 5, max_batch=5, nnz_capacity=nnz0 + 2000,
                          init_iters=iters)
    cols, vd = lib.coo_to_device(idx0, v0)
    gpu = lib.Tensor.init_coo(cfg, cols, vd, len(v0), I, J, K0)
    torch.cuda.synchronize()
    A, B, C, lam = gpu.get_factors()
    assert_close(lam, ora.lam, RT, AT, "lambda")
    assert_close(A, ora.A, RT, AT, "A")
    assert_close(B, ora.B, RT, AT, "B")
    assert_close(C, ora.C, RT, AT, "C")
    assert abs(gpu.fit() - ora.fit()) < 1e-5
    gpu.close()
