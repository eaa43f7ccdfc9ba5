"""Parity of the HIP update path with the CPU FP64 oracle (dense tensors).

Bar: sampled indices bit-exact; FP64 path within 1e-8 of the oracle on every
intermediate; FP32 path MTTKRP relative error <= 1e-5 and final fit within 1e-3.
"""

import numpy as np
import pytest

import synth
from oracle import cp
from oracle import sambaten as osb
from parity import assert_close

# FP32 and BF16 paths against the oracle: factor entries within 1e-3 of the
# entry plus 1e-3 of their column's largest entry (the fit bar of 1e-3
# carried to the factors); sampled indices and matchings exact
RT, AT = 1e-3, 1e-3

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def run_pair(lib, I, J, K0, Kn, R, reps, iters, s, seed, prec, batches=1, init="oracle",
             schedule=None, noise=0.01, oracle_bf16=False):
    """Oracle and GPU side by side on one synthetic tensor; yields per-batch debug.
    oracle_bf16: the oracle rounds its summaries to bfloat16 as the BF16 path does."""
    torch = _torch()
    dtype = np.float64 if prec == lib.SBT_P_F64 else np.float32
    gen = synth.DenseCP(I, J, K0 + batches * Kn, R, seed=seed, noise=noise, dtype=dtype)
    X = gen.slices(0, K0 + batches * Kn)
    ocfg = osb.Config(rank=R, reps=reps, als_iters=iters, sample_factor=s, seed=seed,
                      k_capacity=K0 + batches * Kn, init_iters=60, summary_bf16=oracle_bf16)
    if init == "oracle":
        ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X[:, :, :K0])
    else:
        ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X[:, :, :K0],
                               factors=gen.true_model_prefix(K0))
    cfg = lib.make_config(R, reps, iters, s, seed, precision=prec, k_capacity=K0 + batches * Kn,
                          max_batch=Kn, init_iters=60,
                          schedule=lib.SBT_SCHED_BATCHED if schedule is None else schedule)
    gpu = lib.Tensor.init_dense(cfg, lib.dense_to_device(X[:, :, :K0], dtype), I, J, K0,
                                factors=(ora.A, ora.B, ora.C, ora.lam))
    out = []
    for b in range(batches):
        Y = X[:, :, K0 + b * Kn:K0 + (b + 1) * Kn]
        d = ora.update(Y, debug=True)
        gpu.update_batch_dense(lib.dense_to_device(Y, dtype), Kn)
        torch.cuda.synchronize()
        out.append(d)
    return ora, gpu, out


def check_samples(gpu, d, reps):
    for rho in range(reps):
        for mode, key in enumerate(("Is", "Js", "Ks")):
            got = gpu.last_sample(rho, mode)
            np.testing.assert_array_equal(got, d["reps"][rho][key],
                                          err_msg=f"rep {rho} mode {mode}")


def check_reps(lib, gpu, d, reps, rtol, atol):
    """Every repetition's matching exactly, its summary factors A', C', its
    matched A~ and its least-squares rows C~ element by element."""
    for rho in range(reps):
        r = d["reps"][rho]
        np.testing.assert_array_equal(gpu.last_rep(rho, lib.SBT_REP_PI, 1)[0], r["pi"],
                                      err_msg=f"rep {rho}")
        for item, key in ((lib.SBT_REP_AP, "Ap"), (lib.SBT_REP_CP, "Cp"),
                          (lib.SBT_REP_AT, "At"), (lib.SBT_REP_CT, "Ct")):
            assert_close(gpu.last_rep(rho, item, len(r[key])), r[key], rtol, atol,
                         f"{key} rep {rho}")


def test_c1_fp64_update_matches_oracle(lib):
    # 50 x 50 x 40 + one batch of 10, R = 5, s = 2, r = 4, 20 ALS sweeps
    reps, R = 4, 5
    ora, gpu, ds = run_pair(lib, 50, 50, 40, 10, R, reps, 20, 2, 1, lib.SBT_P_F64)
    d = ds[0]
    check_samples(gpu, d, reps)
    n1, n2, Kp = 25, 25, 20 + 10
    for rho in range(reps):
        r = d["reps"][rho]
        np.testing.assert_allclose(gpu.last_rep(rho, lib.SBT_REP_AP, n1), r["Ap"], rtol=1e-8,
                                   atol=1e-10)
        np.testing.assert_allclose(gpu.last_rep(rho, lib.SBT_REP_BP, n2), r["Bp"], rtol=1e-8,
                                   atol=1e-10)
        np.testing.assert_allclose(gpu.last_rep(rho, lib.SBT_REP_CP, Kp), r["Cp"], rtol=1e-8,
                                   atol=1e-10)
        np.testing.assert_allclose(gpu.last_rep(rho, lib.SBT_REP_LAMP, 1)[0], r["lamp"],
                                   rtol=1e-8)
        np.testing.assert_array_equal(gpu.last_rep(rho, lib.SBT_REP_PI, 1)[0], r["pi"])
        np.testing.assert_allclose(gpu.last_rep(rho, lib.SBT_REP_AT, n1), r["At"], rtol=1e-8,
                                   atol=1e-10)
        np.testing.assert_allclose(gpu.last_rep(rho, lib.SBT_REP_CT, Kp), r["Ct"], rtol=1e-7,
                                   atol=1e-9)
    A, B, C, lam = gpu.get_factors()
    np.testing.assert_allclose(C, ora.C, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(A, ora.A, rtol=1e-9, atol=1e-12)
    np.testing.assert_array_equal(lam, ora.lam)
    assert abs(gpu.fit() - ora.fit()) < 1e-9
    assert gpu.batch_counter() == 1 and gpu.shape() == (50, 50, 50, R)


def test_fp64_three_batches_ragged_shapes(lib):
    # sizes that are not multiples of any tile, several batches, K_new = 7
    reps = 3
    ora, gpu, ds = run_pair(lib, 37, 29, 23, 7, 3, reps, 12, 3, 5, lib.SBT_P_F64, batches=3)
    check_samples(gpu, ds[-1], reps)
    _, _, C, _ = gpu.get_factors()
    np.testing.assert_allclose(C, ora.C, rtol=1e-7, atol=1e-9)
    assert abs(gpu.fit() - ora.fit()) < 1e-9


@pytest.mark.parametrize("prec", [0, 1])
def test_twelve_updates_track_the_oracle(lib, prec):
    # Alg. 1 applied again and again: samples exact at every update, the fit
    # after every update and the whole model at the end element by element
    # (FP64 at 1e-8, FP32 at the FP32 bars)
    torch = _torch()
    I, J, K0, Kn, R, reps, nb = 40, 36, 30, 5, 4, 4, 12
    dtype = np.float64 if prec == lib.SBT_P_F64 else np.float32
    gen = synth.DenseCP(I, J, K0 + nb * Kn, R, seed=71, noise=0.01, dtype=dtype)
    X = gen.slices(0, K0 + nb * Kn)
    ocfg = osb.Config(rank=R, reps=reps, als_iters=12, sample_factor=2, seed=71,
                      k_capacity=K0 + nb * Kn)
    ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X[:, :, :K0],
                           factors=gen.true_model_prefix(K0))
    cfg = lib.make_config(R, reps, 12, 2, 71, precision=prec, k_capacity=K0 + nb * Kn,
                          max_batch=Kn)
    gpu = lib.Tensor.init_dense(cfg, lib.dense_to_device(X[:, :, :K0], dtype), I, J, K0,
                                factors=(ora.A, ora.B, ora.C, ora.lam))
    ftol = 1e-9 if prec == lib.SBT_P_F64 else 1e-3
    for b in range(nb):
        Y = X[:, :, K0 + b * Kn:K0 + (b + 1) * Kn]
        d = ora.update(Y, debug=True)
        gpu.update_batch_dense(lib.dense_to_device(Y, dtype), Kn)
        torch.cuda.synchronize()
        check_samples(gpu, d, reps)
        assert abs(gpu.fit() - ora.fit()) < ftol, (b, gpu.fit(), ora.fit())
    A, B, C, lam = gpu.get_factors()
    if prec == lib.SBT_P_F64:
        for got, want in ((A, ora.A), (B, ora.B), (C, ora.C)):
            np.testing.assert_allclose(got, want, rtol=1e-8, atol=1e-10)
        np.testing.assert_allclose(lam, ora.lam, rtol=1e-8)
    else:
        for got, want, name in ((A, ora.A, "A"), (B, ora.B, "B"), (C, ora.C, "C")):
            assert_close(got, want, RT, AT, name)
    assert gpu.batch_counter() == nb


def test_fp32_update_matches_oracle(lib):
    # FP32 store and MTTKRP, FP64 solves; ten repetitions as in the 500^3 workload
    reps = 10
    ora, gpu, ds = run_pair(lib, 100, 90, 60, 12, 10, reps, 30, 5, 2, lib.SBT_P_F32,
                            batches=2, init="true")
    check_samples(gpu, ds[-1], reps)
    check_reps(lib, gpu, ds[-1], reps, RT, AT)
    A, B, C, _ = gpu.get_factors()
    assert abs(gpu.fit() - ora.fit()) < 1e-3
    assert_close(C[60:], ora.C[60:], RT, AT, "new rows of C")
    assert_close(A, ora.A, RT, AT, "A")
    assert_close(B, ora.B, RT, AT, "B")


def test_plain_schedule_matches_batched(lib):
    # same arithmetic, different launch structure and reduction order
    torch = _torch()
    res, samples = [], []
    for sched in (lib.SBT_SCHED_BATCHED, lib.SBT_SCHED_PLAIN):
        ora, gpu, ds = run_pair(lib, 40, 30, 20, 5, 4, 3, 8, 2, 11, lib.SBT_P_F32, init="true",
                                schedule=sched)
        res.append(gpu.get_factors())
        samples.append([gpu.last_sample(r, m) for r in range(3) for m in range(3)])
        torch.cuda.synchronize()
    for a, b in zip(samples[0], samples[1]):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(res[0], res[1]):
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-6)


def test_singleton_batch_and_unit_sample_factor(lib):
    # K_new = 1 (singleton batches, Sec. 3.1) and s = 1 (summary = whole tensor)
    reps = 2
    ora, gpu, ds = run_pair(lib, 12, 10, 6, 1, 2, reps, 10, 1, 3, lib.SBT_P_F64, batches=2,
                            init="true")
    check_samples(gpu, ds[-1], reps)
    np.testing.assert_array_equal(gpu.last_sample(0, 0), np.arange(12))
    _, _, C, _ = gpu.get_factors()
    np.testing.assert_allclose(C, ora.C, rtol=1e-7, atol=1e-9)


def test_init_cp_als_matches_oracle(lib):
    torch = _torch()
    I, J, K0, R = 30, 25, 20, 3
    gen = synth.DenseCP(I, J, K0 + 5, R, seed=9, dtype=np.float64)
    X = gen.slices(0, K0)
    ocfg = osb.Config(rank=R, reps=2, als_iters=5, sample_factor=2, seed=9, k_capacity=K0 + 5,
                      init_iters=50)
    ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X)
    cfg = lib.make_config(R, 2, 5, 2, 9, precision=lib.SBT_P_F64, k_capacity=K0 + 5,
                          max_batch=5, init_iters=50)
    gpu = lib.Tensor.init_dense(cfg, lib.dense_to_device(X, np.float64), I, J, K0)
    torch.cuda.synchronize()
    A, B, C, lam = gpu.get_factors()
    np.testing.assert_allclose(lam, ora.lam, rtol=1e-8)
    np.testing.assert_allclose(A, ora.A, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(C, ora.C, rtol=1e-7, atol=1e-9)
    assert abs(gpu.fit() - ora.fit()) < 1e-10


@pytest.mark.parametrize("I,J,K0,R", [(300, 270, 260, 3), (600, 500, 8, 20)])
def test_init_cp_als_long_factors(lib, I, J, K0, R):
    """Initial CP-ALS where every factor has more rows than one block reduces
    (chunked cross products), and where the two slice factors are too wide for
    the batched mode-3 kernel (the per-step schedule takes over)."""
    torch = _torch()
    gen = synth.DenseCP(I, J, K0 + 2, R, seed=13, dtype=np.float64)
    X = gen.slices(0, K0)
    ocfg = osb.Config(rank=R, reps=1, als_iters=2, sample_factor=2, seed=13, k_capacity=K0 + 2,
                      init_iters=8)
    ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X)
    cfg = lib.make_config(R, 1, 2, 2, 13, precision=lib.SBT_P_F64, k_capacity=K0 + 2,
                          max_batch=2, init_iters=8)
    gpu = lib.Tensor.init_dense(cfg, lib.dense_to_device(X, np.float64), I, J, K0)
    torch.cuda.synchronize()
    A, B, C, lam = gpu.get_factors()
    np.testing.assert_allclose(lam, ora.lam, rtol=1e-8)
    np.testing.assert_allclose(A, ora.A, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(B, ora.B, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(C, ora.C, rtol=1e-6, atol=1e-9)
    assert abs(gpu.fit() - ora.fit()) < 1e-10


def test_numeric_error_leaves_state_unchanged(lib):
    torch = _torch()
    I, J, K0, Kn, R = 16, 14, 10, 4, 2
    gen = synth.DenseCP(I, J, K0 + 2 * Kn, R, seed=4, dtype=np.float32)
    X = gen.slices(0, K0 + 2 * Kn)
    cfg = lib.make_config(R, 2, 5, 2, 4, precision=lib.SBT_P_F32, k_capacity=K0 + 2 * Kn,
                          max_batch=Kn)
    gpu = lib.Tensor.init_dense(cfg, lib.dense_to_device(X[:, :, :K0], np.float32), I, J, K0,
                                factors=gen.true_model_prefix(K0))
    before = gpu.get_factors()
    Y = X[:, :, K0:K0 + Kn].copy()
    Y[3, 2, 1] = np.nan
    st = gpu.try_update_batch_dense(lib.dense_to_device(Y, np.float32), Kn)
    assert st == lib.SBT_E_NUMERIC
    after = gpu.get_factors()
    for a, b in zip(before, after):
        np.testing.assert_array_equal(a, b)
    assert gpu.shape()[2] == K0 and gpu.batch_counter() == 0
    # shape errors: empty batch, over max_batch
    assert gpu.try_update_batch_dense(lib.dense_to_device(Y, np.float32), 0) == lib.SBT_E_SHAPE
    assert gpu.try_update_batch_dense(lib.dense_to_device(Y, np.float32), Kn + 1) == lib.SBT_E_SHAPE
    # the next good batch still goes through, with the counter that was not consumed
    gpu.update_batch_dense(lib.dense_to_device(X[:, :, K0:K0 + Kn], np.float32), Kn)
    torch.cuda.synchronize()
    assert gpu.shape()[2] == K0 + Kn and gpu.batch_counter() == 1


def bf16_round(x):
    """float32 values rounded to the nearest bfloat16 (ties to even), as
    (uint16 bits, float64 values)."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    bits = r.astype(np.uint16)
    vals = (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return bits, vals


@pytest.mark.parametrize("prec,tol,sched", [(0, 1e-12, 0), (0, 1e-12, 1), (1, 1e-5, 0),
                                             (1, 1e-5, 1), (2, 1e-2, 0)])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_mttkrp_kernel_relative_error(lib, prec, tol, sched, mode):
    # BF16 (prec 2) runs the matrix-core kernels: n1 = 97 exercises the padding
    torch = _torch()
    g = np.random.default_rng(100 + mode)
    n1, n2, n3, R = 97, 61, 45, 10
    Z = g.random((n1, n2, n3))
    U = [g.random((n, R)) for n in (n1, n2, n3)]
    if prec == 2:
        bits, Zr = bf16_round(Z)
        Zd = torch.from_numpy(np.ascontiguousarray(bits.transpose(2, 1, 0)).view(np.int16)).cuda()
    else:
        dtype = np.float64 if prec == 0 else np.float32
        Zd = lib.dense_to_device(Z, dtype)
        Zr = Z.astype(dtype).astype(np.float64)
    Ud = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in U]
    out = torch.zeros((Z.shape[mode], R), dtype=torch.float64, device="cuda")
    lib.mttkrp_dense(prec, Zd, n1, n2, n3, R, Ud[0], Ud[1], Ud[2], mode, out, schedule=sched)
    torch.cuda.synchronize()
    ref = cp.mttkrp_dense(Zr, U, mode)
    got = out.cpu().numpy()
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= tol, rel
    assert_close(got, ref, tol, tol / 10, f"mode {mode}")


@pytest.mark.parametrize("R", [5, 20])
def test_mttkrp_bf16_rank_tiles(lib, R):
    # one (R <= 16) and two (R > 16) column tiles of the matrix-core kernels
    torch = _torch()
    g = np.random.default_rng(300 + R)
    n1, n2, n3 = 40, 33, 70
    Z = g.random((n1, n2, n3))
    U = [g.random((n, R)) for n in (n1, n2, n3)]
    bits, Zr = bf16_round(Z)
    Zd = torch.from_numpy(np.ascontiguousarray(bits.transpose(2, 1, 0)).view(np.int16)).cuda()
    Ud = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in U]
    for mode in range(3):
        out = torch.zeros((Z.shape[mode], R), dtype=torch.float64, device="cuda")
        lib.mttkrp_dense(2, Zd, n1, n2, n3, R, Ud[0], Ud[1], Ud[2], mode, out)
        torch.cuda.synchronize()
        ref = cp.mttkrp_dense(Zr, U, mode)
        rel = np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref)
        assert rel <= 1e-2, (mode, rel)


@pytest.mark.parametrize("R", [5, 20])
def test_mttkrp_bf16_long_third_mode(lib, R):
    # a third mode longer than one LDS chunk of C~ in the matrix-core pass W
    # (992 columns at R <= 16, 480 above): n3 = 1100 takes two and three chunks
    torch = _torch()
    g = np.random.default_rng(400 + R)
    n1, n2, n3 = 24, 21, 1100
    Z = g.random((n1, n2, n3))
    U = [g.random((n, R)) for n in (n1, n2, n3)]
    bits, Zr = bf16_round(Z)
    Zd = torch.from_numpy(np.ascontiguousarray(bits.transpose(2, 1, 0)).view(np.int16)).cuda()
    Ud = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in U]
    for mode in range(3):
        out = torch.zeros((Z.shape[mode], R), dtype=torch.float64, device="cuda")
        lib.mttkrp_dense(2, Zd, n1, n2, n3, R, Ud[0], Ud[1], Ud[2], mode, out)
        torch.cuda.synchronize()
        ref = cp.mttkrp_dense(Zr, U, mode)
        got = out.cpu().numpy()
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert rel <= 1e-2, (mode, rel)
        assert_close(got, ref, 1e-2, 1e-3, f"mode {mode}")


def test_bf16_update_with_long_summaries(lib):
    # s = 2 over 1000 old slices: K' = 500 + 10 = 510, then 505 + 10 = 515
    # summary slices at R = 20, past one chunk (480 columns) of the matrix-core
    # pass W staging
    reps = 2
    ora, gpu, ds = run_pair(lib, 40, 36, 1000, 10, 20, reps, 8, 2, 13, lib.SBT_P_BF16,
                            batches=2, init="true", oracle_bf16=True)
    check_samples(gpu, ds[-1], reps)
    assert len(ds[-1]["reps"][0]["Ks"]) + 10 > 480
    A, _, C, _ = gpu.get_factors()
    assert abs(gpu.fit() - ora.fit()) < 1e-4
    assert_close(C[1000:], ora.C[1000:], RT, AT, "new rows of C")
    assert_close(A, ora.A, RT, AT, "A")


def test_bf16_update_matches_oracle(lib):
    # BF16 summaries on the matrix cores, FP64 solves.  Bars: samples bit-exact;
    # fit within 1e-3 of the FP64 oracle; new rows of C within 1e-3 of the
    # oracle that rounds its summaries to BF16 the same way (the new rows
    # themselves move by a few percent between FP64 and BF16 summaries: the
    # summary ALS is ill conditioned for non-negative factors, the fit is not)
    reps = 10
    args = (100, 90, 60, 12, 10, reps, 30, 5, 2, lib.SBT_P_BF16)
    ora16, gpu, ds = run_pair(lib, *args, batches=2, init="true", oracle_bf16=True)
    check_samples(gpu, ds[-1], reps)
    check_reps(lib, gpu, ds[-1], reps, RT, AT)
    ora64, gpu64, _ = run_pair(lib, *args, batches=2, init="true")
    A, _, C, _ = gpu.get_factors()
    assert abs(gpu.fit() - ora64.fit()) < 1e-3
    assert abs(gpu.fit() - ora16.fit()) < 1e-4
    assert_close(C[60:], ora16.C[60:], RT, AT, "new rows of C")
    assert_close(A, ora16.A, RT, AT, "A")


def test_bf16_rank20_ragged_update(lib):
    # two column tiles, n1 not a multiple of 8, K' not a multiple of 32
    reps = 4
    ora, gpu, ds = run_pair(lib, 90, 76, 40, 9, 20, reps, 15, 3, 8, lib.SBT_P_BF16,
                            batches=2, init="true", oracle_bf16=True)
    check_samples(gpu, ds[-1], reps)
    assert abs(gpu.fit() - ora.fit()) < 1e-3


def test_zero_entries_filled_from_the_repetitions(lib):
    # Alg. 1 updates only the zero entries of A, B and of the sampled old rows
    # of C.  Exact zeros are planted in the given model: scattered entries of
    # A, B and C (some in rows that get sampled, some not) and the whole of
    # column 2 of A, whose anchor rows are then zero in every repetition, so
    # no repetition is valid for it: its new rows stay zero and its zeros are
    # not filled.  FP64, element by element against the oracle.
    torch = _torch()
    I, J, K0, Kn, R, reps = 40, 36, 30, 6, 4, 3
    gen = synth.DenseCP(I, J, K0 + Kn, R, seed=31, dtype=np.float64)
    X = gen.slices(0, K0 + Kn)
    A, B, C, lam = (np.array(m) for m in gen.true_model_prefix(K0))
    g = np.random.default_rng(31)
    for M in (A, B, C):
        rows = g.choice(M.shape[0], size=12, replace=False)
        M[rows, g.integers(0, R, 12)] = 0.0
    A[:, 2] = 0.0
    ocfg = osb.Config(rank=R, reps=reps, als_iters=15, sample_factor=2, seed=31,
                      k_capacity=K0 + Kn)
    ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X[:, :, :K0], factors=(A, B, C, lam))
    cfg = lib.make_config(R, reps, 15, 2, 31, precision=lib.SBT_P_F64, k_capacity=K0 + Kn,
                          max_batch=Kn)
    gpu = lib.Tensor.init_dense(cfg, lib.dense_to_device(X[:, :, :K0], np.float64), I, J, K0,
                                factors=(A, B, C, lam))
    d = ora.update(X[:, :, K0:], debug=True)
    gpu.update_batch_dense(lib.dense_to_device(X[:, :, K0:], np.float64), Kn)
    torch.cuda.synchronize()
    check_samples(gpu, d, reps)
    for rho in range(reps):
        assert not d["reps"][rho]["valid"][2]
        np.testing.assert_array_equal(gpu.last_rep(rho, lib.SBT_REP_VALID, 1)[0].astype(bool),
                                      d["reps"][rho]["valid"])
    Ag, Bg, Cg, lg = gpu.get_factors()
    # the oracle did fill zeros: some in sampled rows changed, unsampled ones stayed
    sampled_a = np.unique(np.concatenate([d["reps"][q]["Is"] for q in range(reps)]))
    filled = (A == 0.0) & (ora.A != 0.0)
    assert filled.any() and np.all(np.isin(np.nonzero(filled)[0], sampled_a))
    assert np.any((A == 0.0) & ~np.isin(np.arange(I), sampled_a)[:, None])
    assert (C == 0.0).sum() > (ora.C[:K0] == 0.0).sum()
    assert np.all(ora.A[:, 2] == 0.0) and np.all(ora.C[K0:, 2] == 0.0)
    np.testing.assert_allclose(Ag, ora.A, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Bg, ora.B, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Cg, ora.C, rtol=1e-7, atol=1e-9)
    np.testing.assert_array_equal(Ag == 0.0, ora.A == 0.0)
    np.testing.assert_array_equal(Bg == 0.0, ora.B == 0.0)
    np.testing.assert_array_equal(Cg[:K0] == 0.0, ora.C[:K0] == 0.0)
    assert abs(gpu.fit() - ora.fit()) < 1e-9


def test_full_size_dense500_update(lib):
    # one update of the dense benchmark workload at its full size: 500^3 FP32
    # from a rank-10 U[0,1) model plus 1% noise, 50 new slices, s = 5, r = 10,
    # 30 sweeps, launched as the benchmark launches it (batched FP32).  Every
    # sampled index and every matching exact; the summary factors, the
    # least-squares rows and the grown model element by element; fit within
    # 1e-3 of the FP64 oracle's.
    torch = _torch()
    I = J = K0 = 500
    Kn, R, reps, iters, s = 50, 10, 10, 30, 5
    gen = synth.DenseCP(I, J, K0 + Kn, R, seed=2, noise=0.01, dtype=np.float32)
    Xkji = np.empty((K0 + Kn, J, I), dtype=np.float32)
    gen.fill_slices_kji(Xkji, 0, K0 + Kn)
    X = Xkji.transpose(2, 1, 0)
    model = gen.true_model_prefix(K0)
    ocfg = osb.Config(rank=R, reps=reps, als_iters=iters, sample_factor=s, seed=2,
                      k_capacity=K0 + Kn)
    ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X[:, :, :K0], factors=model)
    cfg = lib.make_config(R, reps, iters, s, 2, precision=lib.SBT_P_F32, k_capacity=K0 + Kn,
                          max_batch=Kn)
    Xd = torch.from_numpy(Xkji).cuda()
    gpu = lib.Tensor.init_dense(cfg, Xd[:K0], I, J, K0, factors=model)
    d = ora.update(X[:, :, K0:], debug=True)
    gpu.update_batch_dense(Xd[K0:], Kn)
    torch.cuda.synchronize()
    check_samples(gpu, d, reps)
    check_reps(lib, gpu, d, reps, RT, AT)
    A, B, C, _ = gpu.get_factors()
    assert_close(C[K0:], ora.C[K0:], RT, AT, "new rows of C")
    np.testing.assert_array_equal(A, ora.A)  # no zero entries: A is kept as it was
    assert abs(gpu.fit() - ora.fit()) < 1e-3


def test_full_size_dense2000_bf16_update(lib):
    # one update of the default benchmark workload at its full size: a
    # 2000 x 2000 x 1000 FP32 store from a rank-20 U[0,1) model plus 1% noise
    # generated on the GPU as the benchmark generates it, 100 new slices,
    # s = 5, r = 10, 30 sweeps, launched as the benchmark launches it (batched,
    # BF16 summaries on the matrix cores).  The oracle reads the same bytes
    # (copied back) and rounds its summaries to BF16 as the path does.  Every
    # sampled index and every matching exact; the new rows of C at the
    # FP32/BF16 bars; fit within 1e-4 of the oracle's.
    import os
    torch = _torch()
    I = J = 2000
    K0, Kn, R, reps, iters, s = 1000, 100, 20, 10, 30, 5
    gen = synth.DenseCP(I, J, K0 + Kn, R, seed=5, noise=0.01, dtype=np.float32)
    Xd = torch.empty((K0 + Kn, J, I), dtype=torch.float32, device="cuda")
    gen.fill_device(torch, Xd)
    torch.cuda.synchronize()
    X = Xd.cpu().numpy().transpose(2, 1, 0)  # (I, J, K), column-major
    model = gen.true_model_prefix(K0)
    ocfg = osb.Config(rank=R, reps=reps, als_iters=iters, sample_factor=s, seed=5,
                      k_capacity=K0 + Kn, summary_bf16=True,
                      workers=max(1, min(16, os.cpu_count() or 1)))
    ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X[:, :, :K0], factors=model)
    cfg = lib.make_config(R, reps, iters, s, 5, precision=lib.SBT_P_BF16, k_capacity=K0 + Kn,
                          max_batch=Kn)
    gpu = lib.Tensor.init_dense(cfg, Xd[:K0], I, J, K0, factors=model)
    d = ora.update(X[:, :, K0:], debug=True)
    gpu.update_batch_dense(Xd[K0:], Kn)
    torch.cuda.synchronize()
    check_samples(gpu, d, reps)
    for rho in range(reps):
        np.testing.assert_array_equal(gpu.last_rep(rho, lib.SBT_REP_PI, 1)[0],
                                      d["reps"][rho]["pi"], err_msg=f"rep {rho}")
    _, _, C, _ = gpu.get_factors()
    assert_close(C[K0:], ora.C[K0:], RT, AT, "new rows of C")
    assert abs(gpu.fit() - ora.fit()) < 1e-4


@pytest.mark.parametrize("prec,sched", [(0, 0), (0, 1), (1, 0), (2, 0)])
def test_lambda_average_reading(lib, prec, sched):
    # SBT_FLAG_LAMBDA_AVG: lambda becomes the average of its previous value and the
    # summaries' matched weights, against the oracle with the same reading; FP64 at
    # rounding level, FP32 and BF16 (against the BF16-summary oracle) at 1e-3; the
    # given weights are off by a factor so that lambda really moves
    torch = _torch()
    I, J, K0, Kn, R, reps = 44, 40, 30, 5, 4, 3
    dtype = np.float64 if prec == 0 else np.float32
    gen = synth.DenseCP(I, J, K0 + 2 * Kn, R, seed=41, dtype=dtype)
    X = gen.slices(0, K0 + 2 * Kn)
    A, B, C, lam = gen.true_model_prefix(K0)
    lam = lam * np.array([1.5, 0.8, 1.0, 1.2])
    ocfg = osb.Config(rank=R, reps=reps, als_iters=20, sample_factor=2, seed=41,
                      k_capacity=K0 + 2 * Kn, lambda_avg=True, summary_bf16=prec == 2)
    ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X[:, :, :K0], factors=(A, B, C, lam))
    cfg = lib.make_config(R, reps, 20, 2, 41, precision=prec, schedule=sched,
                          k_capacity=K0 + 2 * Kn, max_batch=Kn, flags=lib.SBT_FLAG_LAMBDA_AVG)
    gpu = lib.Tensor.init_dense(cfg, lib.dense_to_device(X[:, :, :K0], dtype), I, J, K0,
                                factors=(A, B, C, lam))
    for b in range(2):
        Y = X[:, :, K0 + b * Kn:K0 + (b + 1) * Kn]
        ora.update(Y)
        gpu.update_batch_dense(lib.dense_to_device(Y, dtype), Kn)
    torch.cuda.synchronize()
    _, _, Cg, lg = gpu.get_factors()
    assert np.abs(lg - lam).max() > 1e-3 * lam.max()  # lambda moved
    tol = 1e-8 if prec == 0 else 1e-3
    np.testing.assert_allclose(lg, ora.lam, rtol=tol)
    assert_close(Cg, ora.C, tol, tol, "C")
    assert abs(gpu.fit() - ora.fit()) < (1e-9 if prec == 0 else 1e-3)
