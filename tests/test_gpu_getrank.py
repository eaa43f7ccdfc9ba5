"""GetRank (Sec. 3.2) on the GPU against the CPU FP64 oracle: the core
consistency of every run, the chosen rank of every summary, the matching of
the R_new sample components and the resulting update."""

import numpy as np
import pytest

import synth
from oracle import sambaten as osb
from parity import assert_close

pytestmark = pytest.mark.gpu


def _pair(lib, I, J, K0, Kn, R_true, R, reps, iters, s, seed, prec, runs, tau, noise=1e-3):
    import torch
    assert torch.cuda.is_available()
    dtype = np.float64 if prec == lib.SBT_P_F64 else np.float32
    gen = synth.DenseCP(I, J, K0 + Kn, R_true, seed=seed, noise=noise, dtype=dtype)
    X = gen.slices(0, K0 + Kn)
    ocfg = osb.Config(rank=R, reps=reps, als_iters=iters, sample_factor=s, seed=seed,
                      k_capacity=K0 + Kn, init_iters=40, getrank_runs=runs,
                      getrank_threshold=tau)
    ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X[:, :, :K0])
    cfg = lib.make_config(R, reps, iters, s, seed, precision=prec, k_capacity=K0 + Kn,
                          max_batch=Kn, getrank_runs=runs, getrank_threshold=tau)
    gpu = lib.Tensor.init_dense(cfg, lib.dense_to_device(X[:, :, :K0], dtype), I, J, K0,
                                factors=(ora.A, ora.B, ora.C, ora.lam))
    d = ora.update(X[:, :, K0:K0 + Kn], debug=True)
    gpu.update_batch_dense(lib.dense_to_device(X[:, :, K0:K0 + Kn], dtype), Kn)
    torch.cuda.synchronize()
    return ora, gpu, d


def _check(lib, ora, gpu, d, reps, R, runs, K0, c_tol, cc_tol, tau=90.0):
    for rho in range(reps):
        r = d["reps"][rho]
        for mode, key in enumerate(("Is", "Js", "Ks")):
            np.testing.assert_array_equal(gpu.last_sample(rho, mode), r[key])
        rn = int(gpu.last_rep(rho, lib.SBT_REP_RNEW, 1, ncols=1)[0, 0])
        assert rn == r["Rnew"], (rho, rn, r["Rnew"], r["cc"])
        cc = gpu.last_rep(rho, lib.SBT_REP_CC, R, ncols=runs)
        want = np.array(r["cc"])
        # Degenerate runs (nearly collinear columns) have core consistencies of
        # -1e3 and below; there the GPU's inverse-Gram form and the oracle's SVD
        # pseudo-inverses differ in value.  Such a score can never reach the
        # threshold on either side (a score is at most 100, and these lie far
        # below any threshold the tests use), so it cannot change the chosen
        # rank: asserted below, and the rest compared in value.
        sane = np.abs(want) < 1e3
        np.testing.assert_allclose(cc[sane], want[sane], rtol=0, atol=cc_tol)
        assert np.all(want[~sane] < 0) and np.all(cc[~sane] < 0)
        assert np.all(want[~sane] < min(tau, 0.0) - 900.0)
        assert np.all(cc[~sane] < min(tau, 0.0) - 900.0)
        valid = gpu.last_rep(rho, lib.SBT_REP_VALID, 1)[0]
        np.testing.assert_array_equal(valid.astype(bool), r["valid"])
        pi = gpu.last_rep(rho, lib.SBT_REP_PI, 1)[0].astype(int)
        m = r["pi"] >= 0
        np.testing.assert_array_equal(pi[m], r["pi"][m])
    A, B, C, lam = gpu.get_factors()
    assert_close(C[K0:], ora.C[K0:], c_tol, c_tol, "new rows of C")
    assert abs(gpu.fit() - ora.fit()) < c_tol


def test_getrank_fp64_rank_deficient_update(lib):
    I, J, K0, Kn, R, reps, runs = 40, 36, 30, 8, 4, 3, 2
    ora, gpu, d = _pair(lib, I, J, K0, Kn, 2, R, reps, 20, 2, 41, lib.SBT_P_F64, runs, 90.0)
    assert all(r["Rnew"] < R for r in d["reps"])
    _check(lib, ora, gpu, d, reps, R, runs, K0, 1e-7, 1e-6)


def test_getrank_fp32(lib):
    I, J, K0, Kn, R, reps, runs = 48, 40, 36, 10, 5, 3, 1
    ora, gpu, d = _pair(lib, I, J, K0, Kn, 3, R, reps, 20, 2, 42, lib.SBT_P_F32, runs, 90.0)
    _check(lib, ora, gpu, d, reps, R, runs, K0, 1e-3, 0.5)


@pytest.mark.parametrize("tau,expect", [(1e9, 1), (-1e308, 3)])
def test_getrank_threshold_edges(lib, tau, expect):
    I, J, K0, Kn, R, reps, runs = 30, 28, 24, 6, 3, 2, 1
    ora, gpu, d = _pair(lib, I, J, K0, Kn, 2, R, reps, 10, 2, 43, lib.SBT_P_F64, runs, tau)
    for rho in range(reps):
        assert d["reps"][rho]["Rnew"] == expect
        assert int(gpu.last_rep(rho, lib.SBT_REP_RNEW, 1, ncols=1)[0, 0]) == expect
    A, B, C, lam = gpu.get_factors()
    assert_close(C[K0:], ora.C[K0:], 1e-7, 1e-7, "new rows of C")


def _pair_coo(lib, I, J, K0, Kn, R_true, R, reps, iters, s, seed, runs, tau):
    import torch
    assert torch.cuda.is_available()
    gen = synth.SparseSupportCP(I, J, K0 + Kn, R_true, seed)
    idx0, v0 = gen.entries(0, K0)
    yi, yv = gen.entries(K0, K0 + Kn)
    nnz = len(v0) + len(yv)
    ocfg = osb.Config(rank=R, reps=reps, als_iters=iters, sample_factor=s, seed=seed,
                      k_capacity=K0 + Kn, nnz_capacity=nnz, init_iters=40, getrank_runs=runs,
                      getrank_threshold=tau)
    ora = osb.OracleTensor(ocfg, osb.COO, (I, J, K0), coo0=(idx0, v0))
    cfg = lib.make_config(R, reps, iters, s, seed, fmt=lib.SBT_COO, precision=lib.SBT_P_F32,
                          k_capacity=K0 + Kn, max_batch=Kn, nnz_capacity=nnz,
                          getrank_runs=runs, getrank_threshold=tau)
    cols, vd = lib.coo_to_device(idx0, v0)
    gpu = lib.Tensor.init_coo(cfg, cols, vd, len(v0), I, J, K0,
                              (ora.A, ora.B, ora.C, ora.lam))
    d = ora.update(coo=(yi, yv, Kn), debug=True)
    bcols, bv = lib.coo_to_device(yi, yv)
    gpu.update_batch_coo(bcols, bv, len(yv), Kn)
    torch.cuda.synchronize()
    return ora, gpu, d


@pytest.mark.parametrize("R,R_true,runs,seed", [(4, 2, 2, 44), (6, 3, 1, 45)])
def test_getrank_coo_summaries(lib, R, R_true, runs, seed):
    # sparse data of exact low rank (factor columns zero on most rows): the
    # COO summaries' CP-ALS runs over their entries and their core
    # consistency is taken slice by slice; FP32 summary arithmetic, so the
    # FP32 bars of the dense test
    I, J, K0, Kn, reps = 44, 40, 30, 8, 3
    ora, gpu, d = _pair_coo(lib, I, J, K0, Kn, R_true, R, reps, 20, 2, seed, runs, 90.0)
    assert all(r["Rnew"] < R for r in d["reps"])
    _check(lib, ora, gpu, d, reps, R, runs, K0, 1e-3, 0.5)


@pytest.mark.parametrize("tau,expect", [(1e9, 1), (-1e308, 3)])
def test_getrank_coo_threshold_edges(lib, tau, expect):
    I, J, K0, Kn, R, reps = 30, 28, 24, 6, 3, 2
    ora, gpu, d = _pair_coo(lib, I, J, K0, Kn, 2, R, reps, 10, 2, 46, 1, tau)
    for rho in range(reps):
        assert d["reps"][rho]["Rnew"] == expect
        assert int(gpu.last_rep(rho, lib.SBT_REP_RNEW, 1, ncols=1)[0, 0]) == expect
    A, B, C, lam = gpu.get_factors()
    assert_close(C[K0:], ora.C[K0:], 1e-3, 1e-3, "new rows of C")
