"""Serving loop: results alone and in a mix of concurrent requests are the
same; admission by staging memory; errors stay with their request."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


SHAPES = [  # (I, J, K0, R, Kn per request, seed)
    (60, 50, 40, 4, (5, 9, 3), 31),
    (80, 40, 30, 6, (7, 2, 11), 32),
    (45, 70, 50, 5, (4, 6, 8), 33),
]


def make(lib, I, J, K0, R, kns, seed, prec):
    torch = _torch()
    Ktot = K0 + sum(kns)
    gen = synth.DenseCP(I, J, Ktot, R, seed=seed, dtype=np.float32)
    X = gen.slices(0, Ktot)
    Xd = lib.dense_to_device(X, np.float32)  # (K, J, I) memory = column-major
    cfg = lib.make_config(R, 4, 12, 2, seed, precision=prec, k_capacity=Ktot,
                          max_batch=max(kns))
    T = lib.Tensor.init_dense(cfg, Xd[:K0], I, J, K0, factors=gen.true_model_prefix(K0))
    batches, k = [], K0
    for kn in kns:
        batches.append(Xd[k:k + kn].clone())
        k += kn
    torch.cuda.synchronize()  # batches complete before the server's streams read them
    return T, batches


@pytest.mark.parametrize("prec", [1, 2])
def test_mix_equals_alone(lib, prec):
    torch = _torch()
    # alone: each tensor's requests applied directly, one after the other
    alone = []
    for I, J, K0, R, kns, seed in SHAPES:
        T, batches = make(lib, I, J, K0, R, kns, seed, prec)
        for Y, kn in zip(batches, kns):
            T.update_batch_dense(Y, kn)
        torch.cuda.synchronize()
        alone.append(T.get_factors())
        T.close()
    # mix: all requests interleaved through a server with 3 slots
    made = [make(lib, I, J, K0, R, kns, seed, prec) for I, J, K0, R, kns, seed in SHAPES]
    srv = lib.Server(3, 64 << 20)
    tickets = []
    for step in range(3):
        for (T, batches), (_, _, _, _, kns, _) in zip(made, SHAPES):
            tickets.append(srv.submit_dense(T, batches[step], kns[step]))
    srv.drain()
    for tk in tickets:
        state, res, ts, t0, t1 = srv.poll(tk)
        assert state == 2 and res == lib.SBT_OK
        assert ts <= t0 <= t1
    for (T, _), ref in zip(made, alone):
        got = T.get_factors()
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
        assert T.batch_counter() == 3
    srv.close()
    for T, _ in made:
        T.close()


def test_admission_by_staging_memory(lib):
    torch = _torch()
    I, J, K0, R, kns, seed = SHAPES[0]
    T, batches = make(lib, I, J, K0, R, kns, seed, 1)
    one = (I * J * max(kns) * 4 + 255) // 256 * 256
    srv = lib.Server(2, one)  # one batch at a time fits
    st, _ = srv.try_submit_dense(T, batches[0], 10 ** 6)  # larger than the pool
    assert st == lib.SBT_E_NOMEM
    T2, b2 = make(lib, *SHAPES[1][:4], SHAPES[1][4], SHAPES[1][5], 1)
    tks = [srv.submit_dense(T, batches[i], kns[i]) for i in range(3)]
    tks += [srv.submit_dense(T2, b2[0], SHAPES[1][4][0])]
    srv.drain()
    for tk in tks:
        assert srv.poll(tk)[:2] == (2, lib.SBT_OK)
    assert T.batch_counter() == 3 and T2.batch_counter() == 1
    srv.close()
    torch.cuda.synchronize()


def test_error_stays_with_its_request(lib):
    torch = _torch()
    (T1, b1), (T2, b2) = [make(lib, I, J, K0, R, kns, seed, 1)
                          for I, J, K0, R, kns, seed in SHAPES[:2]]
    before = T1.get_factors()
    bad = b1[0].clone()
    bad.view(-1)[5] = float("nan")
    torch.cuda.synchronize()
    srv = lib.Server(2, 64 << 20)
    t_bad = srv.submit_dense(T1, bad, SHAPES[0][4][0])
    t_ok = srv.submit_dense(T2, b2[0], SHAPES[1][4][0])
    srv.drain()
    assert srv.poll(t_bad)[:2] == (2, lib.SBT_E_NUMERIC)
    assert srv.poll(t_ok)[:2] == (2, lib.SBT_OK)
    for a, b in zip(T1.get_factors(), before):
        np.testing.assert_array_equal(a, b)
    assert T1.batch_counter() == 0 and T2.batch_counter() == 1
    srv.close()
    torch.cuda.synchronize()


def test_served_tensors_replayed_through_the_oracle(lib):
    # FP64 tensors served with interleaved requests on three slots; each tensor's
    # requests replayed in arrival order through the oracle: samples of the last
    # update bit-exact, model element by element at 1e-7, fit within 1e-9
    from oracle import sambaten as osb
    torch = _torch()
    made, oracles, data = [], [], []
    for q, (I, J, K0, R, kns, seed) in enumerate(SHAPES):
        Ktot = K0 + sum(kns)
        gen = synth.DenseCP(I, J, Ktot, R, seed=seed, dtype=np.float64)
        X = gen.slices(0, Ktot)
        model = gen.true_model_prefix(K0)
        ocfg = osb.Config(rank=R, reps=4, als_iters=12, sample_factor=2, seed=seed,
                          tensor_id=q, k_capacity=Ktot)
        oracles.append(osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=X[:, :, :K0],
                                        factors=model))
        cfg = lib.make_config(R, 4, 12, 2, seed, precision=lib.SBT_P_F64, k_capacity=Ktot,
                              max_batch=max(kns), tensor_id=q)
        Xd = lib.dense_to_device(X, np.float64)
        made.append(lib.Tensor.init_dense(cfg, Xd[:K0], I, J, K0, factors=model))
        data.append((X, Xd))
    torch.cuda.synchronize()
    srv = lib.Server(3, 64 << 20)
    order = []
    g = np.random.default_rng(3)
    pending = [list(kns) for *_, kns, _ in SHAPES]
    pos = [K0 for _, _, K0, *_ in SHAPES]
    while any(pending):
        q = int(g.choice([i for i in range(3) if pending[i]]))
        kn = pending[q].pop(0)
        Xd = data[q][1]
        srv.submit_dense(made[q], Xd[pos[q]:pos[q] + kn], kn)
        order.append((q, pos[q], kn))
        pos[q] += kn
    srv.drain()
    for q, k0, kn in order:  # the oracle in the same per-tensor arrival order
        d = oracles[q].update(data[q][0][:, :, k0:k0 + kn], debug=True)
        if k0 + kn == pos[q]:
            for rho in range(4):
                for mode, key in enumerate(("Is", "Js", "Ks")):
                    np.testing.assert_array_equal(made[q].last_sample(rho, mode),
                                                  d["reps"][rho][key])
    for T, ora in zip(made, oracles):
        A, B, C, lam = T.get_factors()
        np.testing.assert_allclose(A, ora.A, rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(B, ora.B, rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(C, ora.C, rtol=1e-7, atol=1e-9)
        assert abs(T.fit() - ora.fit()) < 1e-9
    srv.close()
    for T in made:
        T.close()
