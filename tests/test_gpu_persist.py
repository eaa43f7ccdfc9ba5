"""Persistent summaries on the GPU against the CPU FP64 oracle: kept sample
indices, periodic redraws and the warm-started summary CP-ALS."""

import numpy as np
import pytest

import synth
from oracle import sambaten as osb
from parity import assert_close

pytestmark = pytest.mark.gpu


def _run(lib, prec, refresh, schedule=None, batches=3, seed=51):
    import torch
    assert torch.cuda.is_available()
    I, J, K0, Kn, R, reps, iters = 40, 36, 30, 6, 3, 3, 20
    dtype = np.float64 if prec == lib.SBT_P_F64 else np.float32
    bf16 = prec == lib.SBT_P_BF16
    gen = synth.DenseCP(I, J, K0 + batches * Kn, R, seed=seed, noise=0.01, dtype=dtype)
    X = gen.slices(0, K0 + batches * Kn)
    ocfg = osb.Config(rank=R, reps=reps, als_iters=iters, sample_factor=2, seed=seed,
                      k_capacity=K0 + batches * Kn, init_iters=40, persist_summaries=True,
                      summary_refresh=refresh, summary_bf16=bf16)
    ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X[:, :, :K0])
    cfg = lib.make_config(R, reps, iters, 2, seed, precision=prec, k_capacity=K0 + batches * Kn,
                          max_batch=Kn, persist_summaries=True, summary_refresh=refresh,
                          schedule=lib.SBT_SCHED_BATCHED if schedule is None else schedule)
    gpu = lib.Tensor.init_dense(cfg, lib.dense_to_device(X[:, :, :K0], dtype), I, J, K0,
                                factors=(ora.A, ora.B, ora.C, ora.lam))
    ds = []
    for b in range(batches):
        Y = X[:, :, K0 + b * Kn:K0 + (b + 1) * Kn]
        d = ora.update(Y, debug=True)
        gpu.update_batch_dense(lib.dense_to_device(Y, dtype), Kn)
        torch.cuda.synchronize()
        for rho in range(reps):
            for mode, key in enumerate(("Is", "Js", "Ks")):
                np.testing.assert_array_equal(gpu.last_sample(rho, mode), d["reps"][rho][key],
                                              err_msg=f"batch {b} rep {rho} mode {mode}")
            if prec == lib.SBT_P_F64:
                # from the third update on the summary sweeps replay a captured
                # graph: every replay is checked
                Ap = gpu.last_rep(rho, lib.SBT_REP_AP, I)
                np.testing.assert_allclose(Ap, d["reps"][rho]["Ap"], rtol=1e-7, atol=1e-9,
                                           err_msg=f"batch {b} rep {rho}")
        ds.append(d)
    return ora, gpu, ds, K0


def test_persistent_fp64_matches_oracle(lib):
    ora, gpu, ds, K0 = _run(lib, lib.SBT_P_F64, 0, batches=5)
    for d in ds[1:]:  # the same anchors every time
        for rho in range(3):
            np.testing.assert_array_equal(d["reps"][rho]["Ks"], ds[0]["reps"][rho]["Ks"])
    A, B, C, lam = gpu.get_factors()
    np.testing.assert_allclose(C[K0:], ora.C[K0:], rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(A, ora.A, rtol=1e-7, atol=1e-9)
    assert abs(gpu.fit() - ora.fit()) < 1e-9
    Bp = gpu.last_rep(0, lib.SBT_REP_BP, 40)
    np.testing.assert_allclose(Bp, ds[-1]["reps"][0]["Bp"], rtol=1e-7, atol=1e-9)


def test_persistent_redraw_every_two_fp32(lib):
    ora, gpu, ds, K0 = _run(lib, lib.SBT_P_F32, 2, batches=4)
    A, B, C, lam = gpu.get_factors()
    # FP32 summaries: entries within 1e-3 of the entry plus 1e-3 of the column's
    # largest (the fit bar carried to the factors)
    assert_close(C[K0:], ora.C[K0:], 1e-3, 1e-3, "new rows of C")
    assert_close(A, ora.A, 1e-3, 1e-3, "A")
    for rho in range(3):
        assert_close(gpu.last_rep(rho, lib.SBT_REP_AP, 40), ds[-1]["reps"][rho]["Ap"], 1e-3,
                     1e-3, f"A' rep {rho}")
    assert abs(gpu.fit() - ora.fit()) < 1e-3


def test_persistent_plain_schedule_fp64(lib):
    ora, gpu, ds, K0 = _run(lib, lib.SBT_P_F64, 0, schedule=lib.SBT_SCHED_PLAIN, batches=2)
    A, B, C, lam = gpu.get_factors()
    np.testing.assert_allclose(C[K0:], ora.C[K0:], rtol=1e-7, atol=1e-9)


def test_persistent_bf16_matrix_cores(lib):
    # the kept summary's old part stays in both BF16 layouts; only the new
    # slices' groups are gathered again
    ora, gpu, ds, K0 = _run(lib, lib.SBT_P_BF16, 0, batches=4)
    A, B, C, lam = gpu.get_factors()
    # against the oracle that rounds its summaries to BF16 the same way
    assert_close(C[K0:], ora.C[K0:], 1e-3, 1e-3, "new rows of C")
    assert_close(A, ora.A, 1e-3, 1e-3, "A")
    for rho in range(3):
        assert_close(gpu.last_rep(rho, lib.SBT_REP_AP, 40), ds[-1]["reps"][rho]["Ap"], 1e-3,
                     1e-3, f"A' rep {rho}")
    assert abs(gpu.fit() - ora.fit()) < 1e-4
