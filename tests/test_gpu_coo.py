"""Parity of the HIP sparse (COO) update path with the CPU FP64 oracle."""

import numpy as np
import pytest

import synth
from oracle import sambaten as osb

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


def test_coo_update_matches_oracle(lib):
    reps = 4
    ora, gpu, ds = run_coo_pair(lib, 80, 70, 40, 10, 2, 3, reps, 15, 2, 21, 6000, 1500)
    d = ds[-1]
    for rho in range(reps):
        for mode, key in enumerate(("Is", "Js", "Ks")):
            np.testing.assert_array_equal(gpu.last_sample(rho, mode), d["reps"][rho][key])
        r = d["reps"][rho]
        Ap = gpu.last_rep(rho, lib.SBT_REP_AP, 40)
        assert np.linalg.norm(Ap - r["Ap"]) <= 1e-3 * np.linalg.norm(r["Ap"])
        np.testing.assert_array_equal(gpu.last_rep(rho, lib.SBT_REP_PI, 1)[0], r["pi"])
    A, B, C, lam = gpu.get_factors()
    err = np.linalg.norm(C[40:] - ora.C[40:]) / np.linalg.norm(ora.C[40:])
    assert err < 1e-3, err
    assert abs(gpu.fit() - ora.fit()) < 1e-3
    assert gpu.shape()[2] == 60


@pytest.mark.parametrize("I,J,K0,R,nnz0,nnz_b", [
    (80, 70, 40, 20, 6000, 1500),    # rank above 16: 32-float factor rows, 8 lanes per entry
    (60, 50, 40, 3, 50000, 6000),    # about 200 summary entries per row: a wavefront per unit
])
def test_coo_update_unit_shapes(lib, I, J, K0, R, nnz0, nnz_b):
    reps = 3
    ora, gpu, ds = run_coo_pair(lib, I, J, K0, 10, 1, R, reps, 10, 2, 23, nnz0, nnz_b)
    d = ds[-1]
    for rho in range(reps):
        for mode, key in enumerate(("Is", "Js", "Ks")):
            np.testing.assert_array_equal(gpu.last_sample(rho, mode), d["reps"][rho][key])
    A, B, C, lam = gpu.get_factors()
    err = np.linalg.norm(C[K0:] - ora.C[K0:]) / np.linalg.norm(ora.C[K0:])
    assert err < 1e-3, err
    assert abs(gpu.fit() - ora.fit()) < 1e-3


def test_coo_persistent_summaries(lib):
    reps = 3
    ora, gpu, ds = run_coo_pair(lib, 80, 70, 40, 10, 3, 3, reps, 12, 2, 25, 6000, 1500,
                                persist=True)
    for rho in range(reps):
        for mode, key in enumerate(("Is", "Js", "Ks")):
            np.testing.assert_array_equal(gpu.last_sample(rho, mode), ds[-1]["reps"][rho][key])
            np.testing.assert_array_equal(ds[-1]["reps"][rho][key], ds[0]["reps"][rho][key])
    A, B, C, lam = gpu.get_factors()
    err = np.linalg.norm(C[40:] - ora.C[40:]) / np.linalg.norm(ora.C[40:])
    assert err < 1e-3, err
    assert abs(gpu.fit() - ora.fit()) < 1e-3


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
