"""Parity of the order-N update of sparse (COO) tensors with the N-mode oracle.

The method is defined on the tensor, not on its storage: the oracle runs on
the same entries as a dense array (every other entry zero, which adds
nothing to the importance sums or to any MTTKRP).  The COO path keeps FP32
values and computes every product and sum in FP64, so the bar is the FP64
one: sampled indices, matchings and validity bit-exact; every per-repetition
intermediate, the model and the fit within 1e-8 relative.
"""

import numpy as np
import pytest

import synth
from oracle import nmode

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def sparse_cp(dims, R, seed, density):
    """A low-rank tensor of FP32 values, thinned to about `density` of its
    entries (the rest exactly zero)."""
    gen = synth.DenseCPN(tuple(dims), R, seed=seed, noise=0.02, dtype=np.float64)
    X = gen.slices(0, dims[-1]).astype(np.float32)
    keep = np.random.default_rng(seed + 7).random(X.shape) < density
    X = np.where(keep, X, np.float32(0.0))
    return X.astype(np.float64), gen


def entries(X, k0, k1):
    """Coordinates (last batch-relative) and values of the nonzeros of slices k0..k1-1."""
    sub = X[..., k0:k1]
    idx = np.argwhere(sub != 0.0)
    return idx.astype(np.int32), sub[tuple(idx.T)].astype(np.float32)


def run_pair(lib, dims, Kn, R, reps, iters, s, seed, batches=2, density=0.35, init="model"):
    torch = _torch()
    N = len(dims)
    K0 = dims[-1]
    Kall = K0 + batches * Kn
    X, gen = sparse_cp(tuple(dims[:-1]) + (Kall,), R, seed, density)
    cfg_o = nmode.Config(rank=R, reps=reps, als_iters=iters, sample_factor=s, seed=seed, order=N,
                         k_capacity=Kall, init_iters=30)
    nnz_all = int(np.count_nonzero(X))
    cfg = lib.make_config(R, reps, iters, 1, seed, fmt=lib.SBT_COO, precision=lib.SBT_P_F32,
                          k_capacity=Kall, max_batch=Kn, nnz_capacity=nnz_all, init_iters=30)
    idx0, v0 = entries(X, 0, K0)
    cols, v = lib.coo_nd_to_device(idx0, v0)
    if init == "model":
        Us, lam = gen.true_model_prefix(K0)
        ora = nmode.OracleTensorN(cfg_o, X[..., :K0], factors=Us, lam=lam)
        gpu = lib.TensorN.init_coo_nd(cfg, cols, v, dims, s, factors=Us, lam=lam)
    else:
        ora = nmode.OracleTensorN(cfg_o, X[..., :K0])
        gpu = lib.TensorN.init_coo_nd(cfg, cols, v, dims, s)
    out = []
    for b in range(batches):
        k0, k1 = K0 + b * Kn, K0 + (b + 1) * Kn
        d = ora.update(X[..., k0:k1], debug=True)
        ib, vb = entries(X, k0, k1)
        cb, vbd = lib.coo_nd_to_device(ib, vb)
        gpu.update_batch_coo_nd(cb, vbd, Kn)
        torch.cuda.synchronize()
        out.append(d)
    return ora, gpu, out, X


def check_update(lib, gpu, ora, d, N, reps, rtol=1e-8, atol=1e-10):
    for rho in range(reps):
        r = d["reps"][rho]
        for m in range(N):
            np.testing.assert_array_equal(gpu.last_sample(rho, m), r["S"][m],
                                          err_msg=f"rep {rho} mode {m}")
        np.testing.assert_array_equal(gpu.last_rep_nd(rho, lib.SBT_ND_REP_PI), r["pi"])
        np.testing.assert_array_equal(gpu.last_rep_nd(rho, lib.SBT_ND_REP_VALID),
                                      r["valid"].astype(float))
        for m in range(N):
            np.testing.assert_allclose(gpu.last_rep_nd(rho, lib.SBT_ND_REP_UP, m), r["Up"][m],
                                       rtol=rtol, atol=atol, err_msg=f"rep {rho} U'_{m}")
        np.testing.assert_allclose(gpu.last_rep_nd(rho, lib.SBT_ND_REP_LAMP), r["lamp"],
                                   rtol=rtol)
        for m in range(N - 1):
            np.testing.assert_allclose(gpu.last_rep_nd(rho, lib.SBT_ND_REP_UT, m), r["Ut"][m],
                                       rtol=rtol, atol=atol, err_msg=f"rep {rho} Ut_{m}")
        np.testing.assert_allclose(gpu.last_rep_nd(rho, lib.SBT_ND_REP_CT), r["Ct"], rtol=rtol,
                                   atol=atol, err_msg=f"rep {rho} Ct")
    Us, lam = gpu.get_factors_nd()
    for m in range(N):
        np.testing.assert_allclose(Us[m], ora.U[m], rtol=rtol, atol=atol, err_msg=f"U_{m}")
    np.testing.assert_allclose(lam, ora.lam, rtol=rtol)


@pytest.mark.parametrize("dims,Kn,R,s,seed", [((14, 12, 10, 16), 4, 3, (2, 3, 2, 2), 41),
                                              ((9, 8, 7, 6, 10), 3, 2, (2, 1, 2, 2, 2), 43),
                                              ((6000, 6, 5, 8), 3, 2, (2, 1, 1, 2), 49)])
def test_coo_update_matches_the_oracle(lib, dims, Kn, R, s, seed):
    # orders 4 and 5, two batches, the generating model given; the last case
    # has 3000 summary rows in mode 0 (three repetitions), so that mode's
    # MTTKRP takes one wavefront per row and the others split their rows
    N, reps = len(dims), 3
    ora, gpu, ds, _ = run_pair(lib, dims, Kn, R, reps, 15, s, seed)
    check_update(lib, gpu, ora, ds[-1], N, reps)
    assert gpu.fit() == pytest.approx(ora.fit(), abs=1e-10)


def test_coo_initial_cp_als_matches_the_oracle(lib):
    # no factors given: CP-ALS on the whole initial tensor, then one batch
    dims, N, reps = (12, 10, 9, 14), 4, 2
    ora, gpu, ds, _ = run_pair(lib, dims, 4, 3, reps, 12, (2, 2, 2, 2), 47, batches=1,
                               init="cp")
    check_update(lib, gpu, ora, ds[-1], N, reps, rtol=1e-7, atol=1e-9)
    assert gpu.fit() == pytest.approx(ora.fit(), abs=1e-9)


def test_coo_empty_batch_and_empty_summaries(lib):
    # a batch with no entry still appends its slices (zero rows); very sparse
    # data leaves some summaries with no entry at all
    torch = _torch()
    dims, N, R, reps = (10, 9, 8, 12), 4, 2, 3
    X, gen = sparse_cp(dims[:-1] + (12 + 2 * 3,), R, 53, 0.04)
    X[..., 12:15] = 0.0  # the first batch is empty
    Us, lam = gen.true_model_prefix(12)
    cfg_o = nmode.Config(rank=R, reps=reps, als_iters=10, sample_factor=(3, 3, 3, 3), seed=53,
                         order=N, k_capacity=18, init_iters=30)
    ora = nmode.OracleTensorN(cfg_o, X[..., :12], factors=Us, lam=lam)
    cfg = lib.make_config(R, reps, 10, 1, 53, fmt=lib.SBT_COO, precision=lib.SBT_P_F32,
                          k_capacity=18, max_batch=3, nnz_capacity=int(np.count_nonzero(X)) + 1)
    i0, v0 = entries(X, 0, 12)
    gpu = lib.TensorN.init_coo_nd(cfg, *lib.coo_nd_to_device(i0, v0), dims, (3, 3, 3, 3),
                                  factors=Us, lam=lam)
    for b in range(2):
        k0 = 12 + 3 * b
        d = ora.update(X[..., k0:k0 + 3], debug=True)
        ib, vb = entries(X, k0, k0 + 3)
        if len(vb) == 0:
            empty = torch.zeros(0, dtype=torch.int32, device="cuda")
            gpu.update_batch_coo_nd([empty] * N, torch.zeros(0, device="cuda"), 3)
        else:
            gpu.update_batch_coo_nd(*lib.coo_nd_to_device(ib, vb), 3)
        torch.cuda.synchronize()
        check_update(lib, gpu, ora, d, N, reps, rtol=1e-7, atol=1e-9)


def test_coo_bad_batches_are_refused_without_change(lib):
    torch = _torch()
    dims, N, R = (8, 7, 6, 10), 4, 2
    X, gen = sparse_cp(dims[:-1] + (14,), R, 59, 0.3)
    Us, lam = gen.true_model_prefix(10)
    cfg = lib.make_config(R, 2, 5, 1, 59, fmt=lib.SBT_COO, precision=lib.SBT_P_F32,
                          k_capacity=14, max_batch=2, nnz_capacity=int(np.count_nonzero(X)))
    i0, v0 = entries(X, 0, 10)
    gpu = lib.TensorN.init_coo_nd(cfg, *lib.coo_nd_to_device(i0, v0), dims, 2, factors=Us,
                                  lam=lam)
    before = gpu.get_factors_nd()
    ib, vb = entries(X, 10, 12)
    out = ib.copy()
    out[0, 1] = 7  # outside mode 1's extent
    with pytest.raises(lib.SbtError):
        gpu.update_batch_coo_nd(*lib.coo_nd_to_device(out, vb), 2)
    late = ib.copy()
    late[0, 3] = 2  # batch-relative last coordinate beyond K_new - 1
    with pytest.raises(lib.SbtError):
        gpu.update_batch_coo_nd(*lib.coo_nd_to_device(late, vb), 2)
    bad = vb.copy()
    bad[1] = np.float32("inf")
    with pytest.raises(lib.SbtError):
        gpu.update_batch_coo_nd(*lib.coo_nd_to_device(ib, bad), 2)
    after = gpu.get_factors_nd()
    for a, b in zip(before[0], after[0]):
        np.testing.assert_array_equal(a, b)
    assert gpu.batch_counter() == 0
    # a good batch still goes through afterwards
    gpu.update_batch_coo_nd(*lib.coo_nd_to_device(ib, vb), 2)
    torch.cuda.synchronize()
    assert gpu.batch_counter() == 1
    # the dense update refuses the COO tensor, and a dense tensor the COO one
    with pytest.raises(lib.SbtError):
        gpu.update_batch_dense(torch.zeros(8 * 7 * 6 * 2, device="cuda"), 2)
