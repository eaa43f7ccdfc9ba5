"""Factor match score on the GPU (sbt_fms) against the CPU FP64 oracle."""

import numpy as np
import pytest

import synth
from oracle import cp
from oracle import sambaten as osb

pytestmark = pytest.mark.gpu


def _tensor(lib, I, J, K0, R, seed, kn=0):
    import torch
    assert torch.cuda.is_available()
    gen = synth.DenseCP(I, J, K0 + max(kn, 1), R, seed=seed, dtype=np.float64)
    X = gen.slices(0, K0 + max(kn, 1))
    g = np.random.default_rng(seed)
    model = tuple(cp.normalize_columns(g.random((n, R)))[0] for n in (I, J, K0)) + (
        g.random(R) + 0.5,)
    cfg = lib.make_config(R, 3, 8, 2, seed, precision=lib.SBT_P_F64, k_capacity=K0 + max(kn, 1),
                          max_batch=max(kn, 1))
    T = lib.Tensor.init_dense(cfg, lib.dense_to_device(X[:, :, :K0], np.float64), I, J, K0,
                              factors=model)
    return T, X, gen


@pytest.mark.parametrize("I,J,K0,R", [(40, 30, 20, 5), (300, 280, 520, 12)])
def test_fms_matches_oracle(lib, I, J, K0, R):
    T, _, _ = _tensor(lib, I, J, K0, R, 31)
    g = np.random.default_rng(32)
    A, B, C, lam = T.get_factors()
    # a reference sharing some components (permuted, rescaled, sign-flipped)
    p = g.permutation(R)
    Ar, Br, Cr = g.random((I, R)), g.random((J, R)), g.random((K0, R))
    Ar[:, : R // 2] = -2.0 * A[:, p[: R // 2]]
    Br[:, : R // 2] = B[:, p[: R // 2]]
    Cr[:, : R // 2] = 0.5 * C[:, p[: R // 2]]
    lr = g.random(R) + 0.2
    got = T.fms(Ar, Br, Cr, lr)
    want = cp.fms(A, B, C, lam, Ar, Br, Cr, lr)
    assert abs(got - want) < 1e-10, (got, want)
    T.close()


def test_fms_of_the_model_itself_is_one(lib):
    T, _, _ = _tensor(lib, 50, 40, 30, 6, 33)
    A, B, C, lam = T.get_factors()
    assert abs(T.fms(A, B, C, lam) - 1.0) < 1e-12
    T.close()


def test_fms_after_update_against_generator(lib):
    """After one update, the score against the generating components (the
    paper's use for synthetic data) equals the oracle's on the same factors."""
    import torch
    I, J, K0, Kn, R = 60, 50, 40, 10, 4
    T, X, gen = _tensor(lib, I, J, K0, R, 34, kn=Kn)
    T.update_batch_dense(lib.dense_to_device(X[:, :, K0:K0 + Kn], np.float64), Kn)
    torch.cuda.synchronize()
    A, B, C, lam = T.get_factors()
    At, Bt, Ct, lt = gen.true_model_prefix(K0 + Kn)
    got = T.fms(At, Bt, Ct, lt)
    want = cp.fms(A, B, C, lam, At, Bt, Ct, lt)
    assert abs(got - want) < 1e-10, (got, want)
    assert 0.0 <= got <= 1.0
    T.close()
