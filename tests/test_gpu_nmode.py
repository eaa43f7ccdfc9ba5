"""Parity of the order-N update (sbt_nd_*) with the N-mode oracle.

Bar: sampled indices and matchings bit-exact; FP64 path within 1e-8 of the
oracle on every per-repetition intermediate and on the model after each
batch; FP32 path (FP32 store and MTTKRP, FP64 everything else) within 1e-3 of
the oracle's fit, the same relative bound as the third-order FP32 path; BF16
path (summaries rounded to BF16, FP32 accumulation) within 1e-3 of the
oracle that rounds its summaries the same way, factor entries and fit.
"""

import numpy as np
import pytest

import synth
from oracle import nmode
from oracle import sambaten as osb
from parity import assert_close

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def run_pair(lib, dims, Kn, R, reps, iters, s, seed, prec, batches=1, init="model", noise=0.02,
             zero=None, oracle_bf16=False):
    """The oracle and the GPU side by side; returns (oracle, gpu, debug per batch).
    oracle_bf16: the oracle rounds its summaries to bfloat16 as the BF16 path does."""
    torch = _torch()
    dtype = np.float64 if prec == lib.SBT_P_F64 else np.float32
    N = len(dims)
    K0 = dims[-1]
    Kall = K0 + batches * Kn
    gen = synth.DenseCPN(tuple(dims[:-1]) + (Kall,), R, seed=seed, noise=noise, dtype=dtype)
    X = gen.slices(0, Kall)
    cfg_o = nmode.Config(rank=R, reps=reps, als_iters=iters, sample_factor=s, seed=seed, order=N,
                         k_capacity=Kall, init_iters=40, summary_bf16=oracle_bf16)
    if init == "model":
        Us, lam = gen.true_model_prefix(K0)
        if zero is not None:
            m, i, f = zero
            Us[m][i, f] = 0.0
        ora = nmode.OracleTensorN(cfg_o, X[..., :K0], factors=Us, lam=lam)
    else:
        ora = nmode.OracleTensorN(cfg_o, X[..., :K0])
    cfg = lib.make_config(R, reps, iters, 1, seed, precision=prec,
                          k_capacity=K0 + max(batches, 1) * Kn, max_batch=Kn, init_iters=40)
    x0 = lib.dense_nd_to_device(X[..., :K0], dtype)
    if init == "model":
        gpu = lib.TensorN.init_dense_nd(cfg, x0, dims, s, factors=Us, lam=lam)
    else:
        gpu = lib.TensorN.init_dense_nd(cfg, x0, dims, s)
    out = []
    for b in range(batches):
        Y = X[..., K0 + b * Kn:K0 + (b + 1) * Kn]
        d = ora.update(Y, debug=True)
        gpu.update_batch_dense(lib.dense_nd_to_device(Y, dtype), Kn)
        torch.cuda.synchronize()
        out.append(d)
    return ora, gpu, out


def check_samples(lib, gpu, d, N, reps):
    for rho in range(reps):
        for m in range(N):
            np.testing.assert_array_equal(gpu.last_sample(rho, m), d["reps"][rho]["S"][m],
                                          err_msg=f"rep {rho} mode {m}")


def check_reps(lib, gpu, d, N, reps, rtol, atol):
    for rho in range(reps):
        r = d["reps"][rho]
        for m in range(N):
            np.testing.assert_allclose(gpu.last_rep_nd(rho, lib.SBT_ND_REP_UP, m), r["Up"][m],
                                       rtol=rtol, atol=atol, err_msg=f"rep {rho} U'_{m}")
        np.testing.assert_allclose(gpu.last_rep_nd(rho, lib.SBT_ND_REP_LAMP), r["lamp"],
                                   rtol=rtol)
        np.testing.assert_array_equal(gpu.last_rep_nd(rho, lib.SBT_ND_REP_PI), r["pi"])
        np.testing.assert_array_equal(gpu.last_rep_nd(rho, lib.SBT_ND_REP_VALID),
                                      r["valid"].astype(float))
        for m in range(N - 1):
            np.testing.assert_allclose(gpu.last_rep_nd(rho, lib.SBT_ND_REP_UT, m), r["Ut"][m],
                                       rtol=rtol, atol=atol, err_msg=f"rep {rho} Ut_{m}")
        np.testing.assert_allclose(gpu.last_rep_nd(rho, lib.SBT_ND_REP_CT), r["Ct"], rtol=rtol,
                                   atol=atol, err_msg=f"rep {rho} Ct")


def check_model(gpu, ora, rtol, atol):
    Us, lam = gpu.get_factors_nd()
    assert len(Us) == ora.N
    for m in range(ora.N):
        np.testing.assert_allclose(Us[m], ora.U[m], rtol=rtol, atol=atol, err_msg=f"U_{m}")
    np.testing.assert_allclose(lam, ora.lam, rtol=rtol)


def test_order3_fp64_matches_oracle(lib):
    # 30 x 28 x 30 + two batches of 5, R = 4, s = (2, 3, 2), r = 3, 15 sweeps
    ora, gpu, ds = run_pair(lib, (30, 28, 30), 5, 4, 3, 15, (2, 3, 2), 5, lib.SBT_P_F64,
                            batches=2)
    check_samples(lib, gpu, ds[-1], 3, 3)
    check_reps(lib, gpu, ds[-1], 3, 3, 1e-8, 1e-10)
    check_model(gpu, ora, 1e-8, 1e-10)
    assert gpu.fit() == pytest.approx(ora.fit(), abs=1e-10)


def test_order4_fp64_matches_oracle(lib):
    # 14 x 12 x 10 x 16 + two batches of 4, R = 3, s = (2, 3, 2, 2), r = 3, 20 sweeps
    N = 4
    ora, gpu, ds = run_pair(lib, (14, 12, 10, 16), 4, 3, 3, 20, (2, 3, 2, 2), 7, lib.SBT_P_F64,
                            batches=2)
    for d in ds[-1:]:
        check_samples(lib, gpu, d, N, 3)
        check_reps(lib, gpu, d, N, 3, 1e-8, 1e-10)
    check_model(gpu, ora, 1e-8, 1e-10)
    assert gpu.shape_nd() == ([14, 12, 10, 24], 3)
    assert gpu.batch_counter() == 2
    assert gpu.fit() == pytest.approx(ora.fit(), abs=1e-10)


def test_order5_fp64_ragged_tiles_and_unit_batch(lib):
    # extents that leave ragged tiles everywhere, a mode sampled whole (s = 1),
    # batches of one slice
    N = 5
    ora, gpu, ds = run_pair(lib, (67, 5, 3, 4, 9), 1, 2, 2, 12, (3, 1, 2, 2, 2), 11,
                            lib.SBT_P_F64, batches=2)
    check_samples(lib, gpu, ds[-1], N, 2)
    check_reps(lib, gpu, ds[-1], N, 2, 1e-8, 1e-10)
    check_model(gpu, ora, 1e-8, 1e-10)


def test_order6_rank1_fp64(lib):
    N = 6
    ora, gpu, ds = run_pair(lib, (5, 3, 4, 2, 3, 8), 3, 1, 2, 10, 2, 13, lib.SBT_P_F64)
    check_samples(lib, gpu, ds[-1], N, 2)
    check_reps(lib, gpu, ds[-1], N, 2, 1e-8, 1e-10)
    check_model(gpu, ora, 1e-8, 1e-10)


def test_order4_initial_cp_als_matches_oracle(lib):
    # no model given: CP-ALS on the whole initial tensor, components by weight
    ora, gpu, ds = run_pair(lib, (12, 11, 9, 14), 3, 3, 2, 10, 2, 17, lib.SBT_P_F64,
                            init="cp", batches=0)
    check_model(gpu, ora, 1e-8, 1e-10)
    assert gpu.fit() == pytest.approx(ora.fit(), abs=1e-10)


def test_order4_middle_modes_beyond_lds_take_the_plain_pass(lib):
    # (0, 70 x 80 merged, last) views of 5600 middle rows: the staged factors
    # of the fused last-mode pass would exceed the 160 KiB of LDS, so the
    # initial CP-ALS, the summary sweeps (s = 1 on the middle modes) and the
    # row solve of the new slices all take the plain pass
    N = 4
    ora, gpu, ds = run_pair(lib, (6, 70, 80, 10), 3, 3, 2, 8, (1, 1, 1, 2), 23, lib.SBT_P_F64,
                            init="cp")
    check_samples(lib, gpu, ds[-1], N, 2)
    check_reps(lib, gpu, ds[-1], N, 2, 1e-8, 1e-10)
    check_model(gpu, ora, 1e-8, 1e-10)
    assert gpu.fit() == pytest.approx(ora.fit(), abs=1e-10)


def test_order4_zero_entry_fill(lib):
    # a zero in the model at an index every repetition samples (s = 1 on mode 1)
    ora, gpu, ds = run_pair(lib, (10, 9, 8, 12), 4, 2, 3, 15, (2, 1, 2, 2), 3, lib.SBT_P_F64,
                            zero=(1, 3, 1))
    check_model(gpu, ora, 1e-8, 1e-10)
    Us, _ = gpu.get_factors_nd()
    assert Us[1][3, 1] != 0.0


def test_order4_fp32_fit_matches_oracle(lib):
    ora, gpu, ds = run_pair(lib, (24, 20, 18, 30), 6, 4, 4, 20, (2, 2, 3, 2), 19, lib.SBT_P_F32,
                            batches=2)
    check_samples(lib, gpu, ds[0] if len(ds) == 1 else ds[-1], 4, 4)
    for rho in range(4):
        np.testing.assert_array_equal(gpu.last_rep_nd(rho, lib.SBT_ND_REP_PI),
                                      ds[-1]["reps"][rho]["pi"])
    f_gpu, f_ora = gpu.fit(), ora.fit()
    assert abs(f_gpu - f_ora) <= 1e-3 * max(1.0, abs(f_ora))
    Us, _ = gpu.get_factors_nd()
    for m in range(4):
        assert_close(Us[m], ora.U[m], 1e-3, 1e-3, f"factor {m}")


@pytest.mark.parametrize("dims,Kn,R,s,seed", [((24, 20, 18, 30), 6, 4, (2, 2, 3, 2), 19),
                                              ((10, 9, 8, 7, 12), 3, 3, (2, 1, 2, 2, 2), 23)])
def test_bf16_summaries_match_the_bf16_oracle(lib, dims, Kn, R, s, seed):
    # orders 4 and 5, two batches: samples and matchings bit-exact; every
    # repetition's summary factors, the model and the fit within 1e-3 of the
    # oracle with BF16 summaries; the fit also within 1e-3 of the FP64 oracle
    N, reps = len(dims), 3
    ora, gpu, ds = run_pair(lib, dims, Kn, R, reps, 20, s, seed, lib.SBT_P_BF16, batches=2,
                            oracle_bf16=True)
    check_samples(lib, gpu, ds[-1], N, reps)
    for rho in range(reps):
        r = ds[-1]["reps"][rho]
        np.testing.assert_array_equal(gpu.last_rep_nd(rho, lib.SBT_ND_REP_PI), r["pi"])
        for m in range(N):
            assert_close(gpu.last_rep_nd(rho, lib.SBT_ND_REP_UP, m), r["Up"][m], 1e-3, 1e-3,
                         f"rep {rho} U'_{m}")
    Us, _ = gpu.get_factors_nd()
    for m in range(N):
        assert_close(Us[m], ora.U[m], 1e-3, 1e-3, f"factor {m}")
    f_gpu, f_ora = gpu.fit(), ora.fit()
    assert abs(f_gpu - f_ora) <= 1e-4 * max(1.0, abs(f_ora))
    ora64, _, _ = run_pair(lib, dims, Kn, R, reps, 20, s, seed, lib.SBT_P_F64, batches=2)
    assert abs(f_gpu - ora64.fit()) <= 1e-3 * max(1.0, abs(ora64.fit()))


def test_non_finite_batch_is_refused_without_change(lib):
    torch = _torch()
    gen = synth.DenseCPN((6, 5, 4, 10), 2, seed=1, noise=0.1, dtype=np.float64)
    X = gen.slices(0, 10)
    Us, lam = gen.true_model_prefix(8)
    cfg = lib.make_config(2, 2, 5, 1, 1, precision=lib.SBT_P_F64, k_capacity=10, max_batch=2)
    gpu = lib.TensorN.init_dense_nd(cfg, lib.dense_nd_to_device(X[..., :8], np.float64),
                                    (6, 5, 4, 8), 2, factors=Us, lam=lam)
    before = gpu.get_factors_nd()
    Y = X[..., 8:].copy()
    Y[2, 1, 3, 0] = np.nan
    with pytest.raises(lib.SbtError) as e:
        gpu.update_batch_dense(lib.dense_nd_to_device(Y, np.float64), 2)
    assert e.value.status == lib.SBT_E_NUMERIC
    torch.cuda.synchronize()
    assert gpu.shape_nd() == ([6, 5, 4, 8], 2)
    after = gpu.get_factors_nd()
    for a, b in zip(before[0], after[0]):
        np.testing.assert_array_equal(a, b)
    # third-order calls are refused on an order-N tensor
    with pytest.raises(lib.SbtError) as e:
        gpu.get_factors()
    assert e.value.status == lib.SBT_E_STATE
    # a batch past the capacity is refused
    Y2 = X[..., 8:]
    with pytest.raises(lib.SbtError):
        gpu.update_batch_dense(lib.dense_nd_to_device(np.concatenate([Y2, Y2], axis=3),
                                                      np.float64), 4)


def test_dense4d_benchmark_configuration(lib):
    """The order-4 benchmark workload at its full size, launched as the
    benchmark launches it (FP32, 120^4 + one batch of 12 slices, R = 10,
    s = 4, r = 10, 30 sweeps), against the oracle's update of the same data:
    every sampled index and every matching exact; per repetition the summary
    lambda and the last-mode rows, and the grown model, element by element
    within 1e-3 of the entry plus 1e-3 of the column's largest entry of the
    FP64 oracle; fits within 1e-3."""
    torch = _torch()
    dims, K0, Kn, R, s, r, iters, seed = (120, 120, 120), 120, 12, 10, 4, 10, 30, 6
    gen = synth.DenseCPN(dims + (K0 + Kn,), R, seed=seed, noise=0.01, dtype=np.float32)
    X = gen.slices(0, K0 + Kn)
    Us, lam = gen.true_model_prefix(K0)
    slice_n = int(np.prod(dims))
    Xd = torch.from_numpy(X.ravel(order="F")).cuda()
    cfg = lib.make_config(R, r, iters, 1, seed, precision=lib.SBT_P_F32, k_capacity=K0 + Kn,
                          max_batch=Kn)
    gpu = lib.TensorN.init_dense_nd(cfg, Xd[:K0 * slice_n], dims + (K0,), s, factors=Us, lam=lam)
    gpu.update_batch_dense(Xd[K0 * slice_n:], Kn)
    torch.cuda.synchronize()
    cfg_o = nmode.Config(rank=R, reps=r, als_iters=iters, sample_factor=s, seed=seed, order=4,
                         k_capacity=K0 + Kn)
    ora = nmode.OracleTensorN(cfg_o, X[..., :K0], factors=Us, lam=lam)
    d = ora.update(X[..., K0:], debug=True)
    check_samples(lib, gpu, d, 4, r)

    for rho in range(r):
        rr = d["reps"][rho]
        np.testing.assert_array_equal(gpu.last_rep_nd(rho, lib.SBT_ND_REP_PI), rr["pi"])
        assert_close(gpu.last_rep_nd(rho, lib.SBT_ND_REP_LAMP), rr["lamp"], 1e-3, 1e-3,
                     f"lambda' rep {rho}")
        assert_close(gpu.last_rep_nd(rho, lib.SBT_ND_REP_CT), rr["Ct"], 1e-3, 1e-3,
                     f"C~ rep {rho}")
    G, _ = gpu.get_factors_nd()
    for m in range(4):
        assert_close(G[m], ora.U[m], 1e-3, 1e-3, f"factor {m}")
    assert abs(gpu.fit() - ora.fit()) < 1e-3


def test_order8_maximum_order_fp64(lib):
    # the largest order the library takes, every extent small
    N = 8
    ora, gpu, ds = run_pair(lib, (3, 2, 3, 2, 2, 3, 2, 6), 2, 2, 2, 8, 1, 23, lib.SBT_P_F64,
                            batches=2)
    check_samples(lib, gpu, ds[-1], N, 2)
    check_reps(lib, gpu, ds[-1], N, 2, 1e-8, 1e-10)
    check_model(gpu, ora, 1e-8, 1e-10)


def test_order4_maximum_rank_fp64(lib):
    # rank 32 (the largest): 32-wide factor rows in every kernel
    N = 4
    ora, gpu, ds = run_pair(lib, (40, 36, 34, 40), 5, 32, 2, 25, (1, 1, 1, 1), 29, lib.SBT_P_F64)
    check_samples(lib, gpu, ds[-1], N, 2)
    check_reps(lib, gpu, ds[-1], N, 2, 1e-7, 1e-9)
    check_model(gpu, ora, 1e-7, 1e-9)


def test_order_and_arguments_refused(lib):
    torch = _torch()
    x = torch.zeros(64, dtype=torch.float64, device="cuda")
    cfg = lib.make_config(2, 2, 5, 1, 1, precision=lib.SBT_P_F64, k_capacity=8, max_batch=2)
    for dims, s in (((4, 4), (1, 1)), ((2,) * 9, (1,) * 9), ((4, 4, 0, 2), (1, 1, 1, 1)),
                    ((4, 4, 2), (1, 0, 1))):
        with pytest.raises(lib.SbtError):
            lib.TensorN.init_dense_nd(cfg, x, dims, s)
    full = lib.make_config(2, 2, 5, 1, 1, precision=lib.SBT_P_F64, k_capacity=2, max_batch=2)
    with pytest.raises(lib.SbtError):  # no room for a batch
        lib.TensorN.init_dense_nd(full, x, (4, 4, 2), (1, 1, 1))
