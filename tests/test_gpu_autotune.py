"""Every launch shape the tuner can pick gives the same update, bit for bit.

The matrix-core path (BF16 summaries) launches its gather and its two MTTKRP
passes in one of three shapes; each output sums the same terms in the same
order in all of them, so the factors after a run of updates must be
identical whatever the shapes, and so must they be while the tuner times the
shapes on the update's own launches and after it has decided.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def run(lib, I, J, K0, Kn, R, reps, iters, s, seed, batches):
    torch = _torch()
    gen = synth.DenseCP(I, J, K0 + batches * Kn, R, seed=seed, noise=0.01, dtype=np.float32)
    X = gen.slices(0, K0 + batches * Kn)
    cfg = lib.make_config(R, reps, iters, s, seed, precision=lib.SBT_P_BF16,
                          k_capacity=K0 + batches * Kn, max_batch=Kn)
    gpu = lib.Tensor.init_dense(cfg, lib.dense_to_device(X[:, :, :K0], np.float32), I, J, K0,
                                factors=gen.true_model_prefix(K0))
    for b in range(batches):
        Y = X[:, :, K0 + b * Kn:K0 + (b + 1) * Kn]
        gpu.update_batch_dense(lib.dense_to_device(Y, np.float32), Kn)
        torch.cuda.synchronize()
    return gpu.get_factors(), gpu.fit()


# n1 n2 = 100 x 90 summary rows (36, 71 or 141 blocks of pass W), K' = 170 to
# 190 (not a multiple of 32), rank 20 (two column tiles) and rank 6 (one)
CASES = [(200, 180, 300, 20, 20, 3, 12, 2, 61), (150, 140, 96, 13, 6, 4, 10, 3, 62)]


@pytest.mark.parametrize("case", CASES)
def test_every_shape_gives_the_same_update(lib, case):
    try:
        ref = None
        for shape in range(lib.SBT_TUNE_SHAPES):
            lib.autotune_set(lib.SBT_TUNE_FIXED, shape)
            got = run(lib, *case, batches=2)
            if ref is None:
                ref = got
                continue
            for a, b, name in zip(got[0], ref[0], "ABCl"):
                np.testing.assert_array_equal(a, b, err_msg=f"shape {shape}: {name}")
            assert got[1] == ref[1]
    finally:
        lib.autotune_set(lib.SBT_TUNE_ON)


def test_online_tuning_decides_and_changes_nothing(lib, tmp_path):
    case = CASES[0]
    try:
        lib.autotune_set(lib.SBT_TUNE_OFF)
        ref = run(lib, *case, batches=3)
        lib.autotune_clear()
        lib.autotune_set(lib.SBT_TUNE_ON)
        got = run(lib, *case, batches=3)
        for a, b, name in zip(got[0], ref[0], "ABCl"):
            np.testing.assert_array_equal(a, b, err_msg=name)
        assert got[1] == ref[1]
        # the two MTTKRP passes are decided after the first update's trials
        # (2 per shape within its 12 sweeps); the gather, once per update,
        # needs six updates of a key
        decided, _ = lib.autotune_count()
        assert decided >= 2
        path = tmp_path / "shapes.txt"
        lib.autotune_save(path)
        rows = [ln.split() for ln in path.read_text().splitlines() if not ln.startswith("#")]
        assert {int(r[1]) for r in rows} >= {1, 2}
        assert all(0 <= int(r[6]) < lib.SBT_TUNE_SHAPES for r in rows)
        # from the file alone, with no trials
        lib.autotune_clear()
        lib.autotune_load(path)
        lib.autotune_set(lib.SBT_TUNE_CACHED)
        again = run(lib, *case, batches=3)
        for a, b, name in zip(again[0], ref[0], "ABCl"):
            np.testing.assert_array_equal(a, b, err_msg=name)
        assert lib.autotune_count() == (len(rows), 0)
    finally:
        lib.autotune_set(lib.SBT_TUNE_ON)
