"""The allocation-free dense MTTKRP entry point against sbt_mttkrp_dense.

Both run the same kernels on the same inputs, so the results must agree to the
bar of each precision's MTTKRP (FP64 1e-12, FP32 1e-5, BF16 1e-2 relative) and,
since the launches are deterministic, they are in fact compared bit for bit.
Two calls in a row go through the one fixed scratch array, the second with a
smaller input, so a stale piece of the first call (the BF16 relayout padding,
a partial row) would show in the second.  Everything goes through the C ABI.
"""

import numpy as np
import pytest

from oracle import cp

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _bf16_bits(x):
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return r.astype(np.uint16), (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _inputs(torch, lib, prec, shape, R, seed):
    g = np.random.default_rng(seed)
    n1, n2, n3 = shape
    Z = g.random(shape)
    U = [g.random((n, R)) for n in shape]
    if prec == lib.SBT_P_BF16:
        bits, Zr = _bf16_bits(Z)
        Zd = torch.from_numpy(np.ascontiguousarray(bits.transpose(2, 1, 0)).view(np.int16)).cuda()
    else:
        dtype = np.float64 if prec == lib.SBT_P_F64 else np.float32
        Zd = lib.dense_to_device(Z, dtype)
        Zr = Z.astype(dtype).astype(np.float64)
    Ud = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in U]
    return Zd, Zr, U, Ud


TOL = {0: 1e-12, 1: 1e-5, 2: 1e-2}


@pytest.mark.parametrize("prec,sched", [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0)])
def test_noalloc_equals_allocating_call_twice(lib, prec, sched):
    torch = _torch()
    stream = torch.cuda.current_stream()
    # the second call is smaller in every extent and in rank
    for call, (shape, R) in enumerate((((97, 61, 45), 20), ((40, 33, 29), 7))):
        Zd, Zr, U, Ud = _inputs(torch, lib, prec, shape, R, 500 + 10 * prec + call)
        for mode in range(3):
            rows = shape[mode]
            ref_out = torch.full((rows, R), np.nan, dtype=torch.float64, device="cuda")
            got = torch.full((rows, R), np.nan, dtype=torch.float64, device="cuda")
            lib.mttkrp_dense(prec, Zd, *shape, R, Ud[0], Ud[1], Ud[2], mode, ref_out,
                             schedule=sched)
            lib.mttkrp_dense_noalloc(prec, Zd, *shape, R, Ud[0], Ud[1], Ud[2], mode, got,
                                     stream=stream, schedule=sched)
            torch.cuda.synchronize()
            a, b = got.cpu().numpy(), ref_out.cpu().numpy()
            assert np.all(np.isfinite(a)), (call, mode)
            ref = cp.mttkrp_dense(Zr, U, mode)
            rel = np.linalg.norm(a - ref) / np.linalg.norm(ref)
            assert rel <= TOL[prec], (call, mode, rel)
            np.testing.assert_allclose(a, b, rtol=TOL[prec], atol=TOL[prec] / 10,
                                       err_msg=f"call {call} mode {mode}")
            assert np.array_equal(a, b), (call, mode, np.abs(a - b).max())


def test_noalloc_enqueues_without_synchronising(lib):
    # three calls queued back to back on one stream, read after one synchronisation:
    # each output equals its own allocating counterpart
    torch = _torch()
    stream = torch.cuda.current_stream()
    shape, R = (64, 50, 30), 10
    Zd, Zr, U, Ud = _inputs(torch, lib, lib.SBT_P_F32, shape, R, 77)
    outs = [torch.zeros((shape[m], R), dtype=torch.float64, device="cuda") for m in range(3)]
    for m in range(3):
        lib.mttkrp_dense_noalloc(lib.SBT_P_F32, Zd, *shape, R, Ud[0], Ud[1], Ud[2], m, outs[m],
                                 stream=stream)
    torch.cuda.synchronize()
    for m in range(3):
        ref_out = torch.zeros((shape[m], R), dtype=torch.float64, device="cuda")
        lib.mttkrp_dense(lib.SBT_P_F32, Zd, *shape, R, Ud[0], Ud[1], Ud[2], m, ref_out)
        torch.cuda.synchronize()
        assert np.array_equal(outs[m].cpu().numpy(), ref_out.cpu().numpy()), m


def test_noalloc_refuses_sizes_beyond_its_array(lib):
    # FP64 mode 0 needs n1 n2 R x 8 bytes of W: 1500 x 1500 x 4 x 8 = 72 MB > 64 MiB.
    # Refused before anything is enqueued (Z is never read, so a small buffer serves).
    torch = _torch()
    R = 4
    Zd = torch.zeros(16, dtype=torch.float64, device="cuda")
    U = [torch.zeros((1500, R), dtype=torch.float64, device="cuda") for _ in range(3)]
    out = torch.zeros((1500, R), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.SbtError) as e:
        lib.mttkrp_dense_noalloc(lib.SBT_P_F64, Zd, 1500, 1500, 2, R, U[0], U[1], U[2], 0, out)
    assert e.value.status == lib.SBT_E_SHAPE
    torch.cuda.synchronize()
    assert float(out.abs().sum()) == 0.0
