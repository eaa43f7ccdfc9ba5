"""The rest of the C ABI around the update (problem statement of Sec. 2.2 and
Algorithm 1's inputs and outputs): checkpoint and resume, one call at a time
per tensor, COO requests and the HBM budget of the serving loop.

Checkpoints: updates applied to a loaded tensor give exactly (bit for bit)
what they give on the tensor that was saved, for dense and COO tensors, with
and without persistent summaries.  Serving: COO requests through a server
equal the same updates applied directly; a budget that holds one request's
working set at a time keeps requests from overlapping; a request larger than
the budget fails alone."""

import os
import threading

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def dense_case(lib, I, J, K0, Kn, batches, R, seed, prec=1, persist=False, reps=4, iters=10,
               s=2):
    torch = _torch()
    Ktot = K0 + batches * Kn
    gen = synth.DenseCP(I, J, Ktot, R, seed=seed, dtype=np.float32)
    X = gen.slices(0, Ktot)
    Xd = lib.dense_to_device(X, np.float32)  # (K, J, I) memory = column-major
    cfg = lib.make_config(R, reps, iters, s, seed, precision=prec, k_capacity=Ktot,
                          max_batch=Kn, persist_summaries=persist)

    def fresh():
        return lib.Tensor.init_dense(cfg, Xd[:K0], I, J, K0, factors=gen.true_model_prefix(K0))

    def apply(T, b):
        T.update_batch_dense(Xd[K0 + b * Kn:K0 + (b + 1) * Kn], Kn)

    torch.cuda.synchronize()
    return fresh, apply


def coo_case(lib, I, J, K0, Kn, batches, R, seed, persist=False, reps=4, iters=10, s=2,
             nnz0=6000, nnz_b=1500):
    gen = synth.SparseCP(I, J, K0 + batches * Kn, R, seed=seed)
    idx0, v0 = gen.slices(0, K0, nnz0, block_id=0)
    bat = [lib.coo_to_device(*gen.slices(K0 + b * Kn, K0 + (b + 1) * Kn, nnz_b, block_id=b + 1))
           for b in range(batches)]
    g = np.random.default_rng(seed)
    A0, B0, C0 = g.random((I, R)), g.random((J, R)), g.random((K0, R))
    nA, nB, nC = (np.linalg.norm(M, axis=0) for M in (A0, B0, C0))
    model = (A0 / nA, B0 / nB, C0 / nC, nA * nB * nC)
    cfg = lib.make_config(R, reps, iters, s, seed, fmt=lib.SBT_COO, precision=lib.SBT_P_F32,
                          k_capacity=K0 + batches * Kn, max_batch=Kn,
                          nnz_capacity=len(v0) + batches * nnz_b, persist_summaries=persist)
    cols, vd = lib.coo_to_device(idx0, v0)

    def fresh():
        return lib.Tensor.init_coo(cfg, cols, vd, len(v0), I, J, K0, model)

    def apply(T, b):
        c, v = bat[b]
        T.update_batch_coo(c, v, int(v.numel()), Kn)

    return fresh, apply, bat


def same_state(lib, T1, T2, reps):
    for a, b in zip(T1.get_factors(), T2.get_factors()):
        np.testing.assert_array_equal(a, b)
    assert T1.batch_counter() == T2.batch_counter()
    assert T1.shape() == T2.shape()
    assert T1.fit() == T2.fit()
    for rho in range(reps):
        for mode in range(3):
            np.testing.assert_array_equal(T1.last_sample(rho, mode), T2.last_sample(rho, mode))


@pytest.mark.parametrize("kind,persist", [("dense", False), ("dense", True), ("bf16", False),
                                          ("coo", False), ("coo", True)])
def test_save_load_resumes_exactly(lib, tmp_path, kind, persist):
    # six updates straight == three, save, destroy, load, three more
    torch = _torch()
    if kind == "coo":
        fresh, apply, _ = coo_case(lib, 60, 50, 40, 6, 6, 4, 71, persist=persist)
    else:
        prec = lib.SBT_P_BF16 if kind == "bf16" else lib.SBT_P_F32
        fresh, apply = dense_case(lib, 48, 40, 30, 5, 6, 4, 72, prec=prec, persist=persist)
    straight = fresh()
    for b in range(6):
        apply(straight, b)
    resumed = fresh()
    for b in range(3):
        apply(resumed, b)
    path = os.path.join(tmp_path, "t.sbt")
    resumed.save(path)
    before = resumed.get_factors()
    resumed.close()
    resumed = lib.Tensor.load_file(path)
    for a, b in zip(resumed.get_factors(), before):
        np.testing.assert_array_equal(a, b)
    assert resumed.batch_counter() == 3
    for b in range(3, 6):
        apply(resumed, b)
    torch.cuda.synchronize()
    same_state(lib, straight, resumed, 4)
    straight.close()
    resumed.close()


def test_load_refuses_bad_files(lib, tmp_path):
    fresh, apply = dense_case(lib, 30, 20, 10, 3, 1, 3, 73)
    T = fresh()
    apply(T, 0)
    good = os.path.join(tmp_path, "good.sbt")
    T.save(good)
    T.close()
    data = open(good, "rb").read()
    cases = {"missing": None, "truncated": data[:-100], "not a checkpoint": b"x" * len(data),
             "header only": data[:512]}
    for name, blob in cases.items():
        path = os.path.join(tmp_path, name.replace(" ", "_"))
        if blob is not None:
            open(path, "wb").write(blob)
        with pytest.raises(lib.SbtError) as e:
            lib.Tensor.load_file(path)
        assert e.value.status == lib.SBT_E_INVALID, name
        assert lib.load().sbt_last_error(None), name
    # the good file still loads
    lib.Tensor.load_file(good).close()


def test_busy_while_a_server_holds_the_tensor(lib):
    # requests queued or running on a server hold their tensor: direct calls are
    # refused with SBT_E_BUSY and change nothing; after the drain they work again
    torch = _torch()
    fresh, apply = dense_case(lib, 300, 280, 200, 40, 4, 10, 74, reps=10, iters=30, s=4)
    T = fresh()
    gen = synth.DenseCP(300, 280, 360, 10, seed=74, dtype=np.float32)
    Xd = lib.dense_to_device(gen.slices(200, 360), np.float32)
    torch.cuda.synchronize()
    srv = lib.Server(1, 64 << 20)
    tks = [srv.submit_dense(T, Xd[40 * b:40 * (b + 1)], 40) for b in range(3)]
    st = T.try_update_batch_dense(Xd[120:160], 40)
    assert st == lib.SBT_E_BUSY
    srv.drain()
    for tk in tks:
        assert srv.poll(tk)[:2] == (2, lib.SBT_OK)
    assert T.batch_counter() == 3
    T.update_batch_dense(Xd[120:160], 40)
    assert T.batch_counter() == 4
    srv.close()
    T.close()


def test_busy_between_host_threads(lib):
    # two host threads on one tensor: each call either runs or returns SBT_E_BUSY,
    # never both at once; the updates that ran are all counted
    torch = _torch()
    fresh, apply = dense_case(lib, 200, 180, 100, 10, 8, 8, 75, reps=10, iters=30, s=4)
    T = fresh()
    gen = synth.DenseCP(200, 180, 180, 8, seed=75, dtype=np.float32)
    Xd = lib.dense_to_device(gen.slices(100, 180), np.float32)
    torch.cuda.synchronize()
    results = []
    lock = threading.Lock()

    def worker(b):
        st = T.try_update_batch_dense(Xd[10 * b:10 * (b + 1)], 10, stream=0)
        with lock:
            results.append(st)

    threads = [threading.Thread(target=worker, args=(b,)) for b in range(8)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    assert set(results) <= {lib.SBT_OK, lib.SBT_E_BUSY}
    assert T.batch_counter() == results.count(lib.SBT_OK) >= 1
    T.close()


def test_coo_requests_through_a_server(lib):
    # COO and dense requests mixed on two slots equal the same updates applied directly
    torch = _torch()
    cases = [coo_case(lib, 60, 50, 40, 6, 3, 4, 76), coo_case(lib, 70, 40, 30, 5, 3, 3, 77)]
    alone = []
    for fresh, apply, _ in cases:
        T = fresh()
        for b in range(3):
            apply(T, b)
        alone.append(T.get_factors())
        T.close()
    dfresh, dapply = dense_case(lib, 40, 36, 20, 4, 3, 3, 78)
    Td = dfresh()
    dref = dfresh()
    for b in range(3):
        dapply(dref, b)
    made = [fresh() for fresh, _, _ in cases]
    srv = lib.Server(2, 64 << 20)
    gen = synth.DenseCP(40, 36, 32, 3, seed=78, dtype=np.float32)
    Xd = lib.dense_to_device(gen.slices(20, 32), np.float32)
    torch.cuda.synchronize()
    tks = []
    for b in range(3):
        for T, (_, _, bat) in zip(made, cases):
            c, v = bat[b]
            tks.append(srv.submit_coo(T, c, v, int(v.numel()), 6 if T is made[0] else 5))
        tks.append(srv.submit_dense(Td, Xd[4 * b:4 * (b + 1)], 4))
    with pytest.raises(lib.SbtError) as e:
        srv.submit_coo(Td, *cases[0][2][0], 10, 6)
    assert e.value.status == lib.SBT_E_STATE
    srv.drain()
    for tk in tks:
        assert srv.poll(tk)[:2] == (2, lib.SBT_OK)
    for T, ref in zip(made, alone):
        for a, b in zip(T.get_factors(), ref):
            np.testing.assert_array_equal(a, b)
    for a, b in zip(Td.get_factors(), dref.get_factors()):
        np.testing.assert_array_equal(a, b)
    srv.close()
    for T in made + [Td, dref]:
        T.close()


def test_hbm_budget_admits_one_working_set_at_a_time(lib):
    # a budget that holds the larger tensor's working set but not two of them: two
    # slots, yet no two requests run at once; a third tensor whose working set
    # exceeds the budget fails alone with SBT_E_NOMEM
    torch = _torch()
    f1, a1 = dense_case(lib, 120, 100, 60, 8, 3, 5, 79, reps=6)
    f2, a2 = dense_case(lib, 110, 90, 50, 8, 3, 5, 80, reps=6)
    f3, _ = dense_case(lib, 300, 300, 40, 8, 1, 8, 81, reps=10, s=1)
    T1, T2, T3 = f1(), f2(), f3()
    ws = [T.memory_bytes()[1] for T in (T1, T2, T3)]
    batch = max(120 * 100, 110 * 90) * 8 * 4
    budget = max(ws[0], ws[1]) + batch + 4096
    assert budget < ws[0] + ws[1] and ws[2] > budget
    g1 = synth.DenseCP(120, 100, 84, 5, seed=79, dtype=np.float32)
    g2 = synth.DenseCP(110, 90, 74, 5, seed=80, dtype=np.float32)
    g3 = synth.DenseCP(300, 300, 48, 8, seed=81, dtype=np.float32)
    Y1 = lib.dense_to_device(g1.slices(60, 84), np.float32)
    Y2 = lib.dense_to_device(g2.slices(50, 74), np.float32)
    Y3 = lib.dense_to_device(g3.slices(40, 48), np.float32)
    torch.cuda.synchronize()
    srv = lib.Server(2, 64 << 20, hbm_budget_bytes=budget)
    tks = []
    for b in range(3):
        tks.append(srv.submit_dense(T1, Y1[8 * b:8 * (b + 1)], 8))
        tks.append(srv.submit_dense(T2, Y2[8 * b:8 * (b + 1)], 8))
    t3 = srv.submit_dense(T3, Y3, 8)
    srv.drain()
    spans = []
    for tk in tks:
        state, res, ts, t0, t1 = srv.poll(tk)
        assert (state, res) == (2, lib.SBT_OK)
        spans.append((t0, t1))
    spans.sort()
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert b0 >= a1, "two working sets ran at once"
    assert srv.poll(t3)[:2] == (2, lib.SBT_E_NOMEM)
    assert T1.batch_counter() == 3 and T2.batch_counter() == 3 and T3.batch_counter() == 0
    srv.close()
    for T in (T1, T2, T3):
        T.close()
